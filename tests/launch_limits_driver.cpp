// Host check of the launch splitting (launch_limits.h): for every element
// count and slab-group count, the launches cover the batch exactly once, in
// order, and none exceeds the workgroup cap or the 2^32 work-item limit of a
// dispatch of 256-thread workgroups.
#include <cstdio>
#include <cstdlib>

#include "launch_limits.h"

static int fails = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::printf("FAIL %s (n=%lld groups=%d)\n", #c, (long long)n, g);  \
      ++fails;                                                           \
    }                                                                    \
  } while (0)

int main() {
  const long long ns[] = {0, 1, 2, 4095, 4096, 50000, (1ll << 22) - 1, 1ll << 22, (1ll << 22) + 1,
                          (1ll << 24) + 12345, 3ll << 25};
  for (long long n : ns) {
    for (int g = 1; g <= 40; ++g) {
      const long long per = dpg::launch_items(g);
      CHECK(per >= 1);
      CHECK(per * g <= dpg::MAX_WG_PER_LAUNCH);
      CHECK(per * g * 256ll < (1ll << 32));
      long long covered = 0, launches = 0;
      for (long long base = 0; base < n; base += per) {
        const long long cnt = (n - base) < per ? (n - base) : per;
        CHECK(base == covered);
        CHECK(cnt >= 1 && cnt * g <= dpg::MAX_WG_PER_LAUNCH);
        covered += cnt;
        ++launches;
      }
      CHECK(covered == n);
      CHECK(launches == dpg::launch_count(n, g));
    }
  }
  std::printf(fails ? "launch limits: %d failures\n" : "launch limits: ok\n", fails);
  return fails ? 1 : 0;
}
