// Host-only stress driver of the serving scheduler, built with the thread or
// address/undefined sanitizers by tests/test_serve_sanitize.py (CPU only: it
// links the scheduler core with its timing stub, never the HIP executor).
//
// Four submitter threads and two pollers race on one server: submits, chunked ones among them (with
// EAGAIN back-off), polls, cancellations of queued requests, releases and
// statistics reads, with a merge limit and a small budget so that admission,
// merging and deferral paths all run.  Exit code 0 = every invariant held.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../include/dpg.h"
#include "../paper_1711_00984_amd/csrc/serve_core.h"
#include "../paper_1711_00984_amd/csrc/terms.h"

using namespace dpg::serve;

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

int main() {
  dpg_serve_cfg cfg{};
  cfg.mem_budget_bytes = int64_t(64) << 20;
  cfg.max_slots = 4096;
  cfg.max_inflight = 16;
  cfg.max_queue = 64;
  cfg.n_streams = 4;
  cfg.max_merge = 8;
  cfg.test_executor = 1;
  cfg.test_fail_launch = 7;
  cfg.test_bytes_per_s = 5e9;
  cfg.test_launch_s = 1e-5;
  CHECK(check_cfg(cfg) == DPG_OK);
  Server srv(cfg, DPG_P_MAX, make_stub_executor(cfg));

  std::vector<double> geom(24 * 256, 0.0);
  std::mutex mu;
  std::vector<uint64_t> live;
  std::atomic<int> submitted{0}, finished{0}, cancelled{0}, failed{0};
  std::atomic<bool> stop{false};
  const int per_thread = 300;

  auto submitter = [&](int seed) {
    std::mt19937 rng(seed);
    for (int i = 0; i < per_thread; ++i) {
      dpg_request r{};
      r.space = int(rng() % 4);
      r.p = 1 + int(rng() % 5);
      r.dp = int(rng() % 2);
      r.prec = int(rng() % 2);
      r.path = DPG_PATH_AUTO;
      r.geom_on_host = 1;
      r.geom.kind = DPG_GEOM_TRILINEAR;
      const int64_t bytes1 = dpg::packed_len(r.space, r.p + r.dp) * (r.prec == DPG_FP32 ? 4 : 8);
      const int64_t nmax = std::min<int64_t>(256, cfg.mem_budget_bytes / 4 / bytes1);
      r.geom.n_elem = 1 + int64_t(rng() % uint64_t(nmax));
      r.geom.data = geom.data();
      r.w0 = r.w1 = 1.0;
      uint64_t t = 0;
      int rc;
      if (i % 5 == 4) {   // a request cut into chunks of at most 3 elements, queued all or none
        r.geom.n_elem = std::min<int64_t>(r.geom.n_elem, 24);
        int64_t k = 0, ce = 0;
        while ((rc = srv.submit_chunked(r, 3 * bytes1, &t, &k, &ce)) == DPG_EAGAIN)
          std::this_thread::sleep_for(std::chrono::microseconds(50));
        CHECK(rc == DPG_OK && t != 0 && ce == 3 && k == (r.geom.n_elem + 2) / 3);
        submitted += int(k);
        std::lock_guard<std::mutex> lk(mu);
        for (int64_t j = 0; j < k; ++j) live.push_back(t + uint64_t(j));
        continue;
      }
      while ((rc = srv.submit(r, &t)) == DPG_EAGAIN) std::this_thread::sleep_for(std::chrono::microseconds(50));
      CHECK(rc == DPG_OK && t != 0);
      ++submitted;
      std::lock_guard<std::mutex> lk(mu);
      live.push_back(t);
    }
  };
  auto poller = [&](int seed) {
    std::mt19937 rng(seed);
    while (!stop.load()) {
      uint64_t t = 0;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (!live.empty()) {
          const size_t k = rng() % live.size();
          t = live[k];
          live[k] = live.back();
          live.pop_back();
        }
      }
      if (!t) {
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        continue;
      }
      dpg_result res{};
      const int rc = srv.poll(t, &res);
      if (rc == DPG_PENDING) {
        if (rng() % 16 == 0 && srv.release(t) == DPG_OK) {   // cancel if still queued
          ++cancelled;
          continue;
        }
        std::lock_guard<std::mutex> lk(mu);
        live.push_back(t);
        continue;
      }
      CHECK(rc == DPG_OK || rc == DPG_EHIP);
      CHECK(res.t_submit <= res.t_admit && res.t_admit <= res.t_done);
      if (rc == DPG_EHIP) ++failed; else ++finished;
      CHECK(srv.release(t) == DPG_OK);
      if (rng() % 8 == 0) {
        dpg_serve_stats st{};
        srv.stats(&st);
        CHECK(st.admitted_bytes <= st.budget_bytes && st.inflight <= cfg.max_inflight);
      }
    }
  };

  std::vector<std::thread> th;
  for (int i = 0; i < 4; ++i) th.emplace_back(submitter, 11 + i);
  std::vector<std::thread> pt;
  for (int i = 0; i < 2; ++i) pt.emplace_back(poller, 101 + i);
  for (auto& x : th) x.join();
  const auto t0 = std::chrono::steady_clock::now();
  while (finished + failed + cancelled < submitted) {
    CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60));
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  stop = true;
  for (auto& x : pt) x.join();

  dpg_serve_stats st{};
  srv.stats(&st);
  CHECK(st.submitted == submitted.load());
  // a request cancelled by the client may have finished between its poll and
  // the release: the server's counts decide which it was
  CHECK(st.completed + st.failed + st.cancelled == st.submitted);
  CHECK(st.completed >= finished.load() && st.failed >= failed.load() && st.cancelled <= cancelled.load());
  CHECK(st.failed >= 1);   // the hooked launch
  CHECK(st.queued == 0 && st.inflight == 0 && st.admitted_bytes == 0);
  CHECK(st.peak_admitted_bytes <= st.budget_bytes);
  std::printf("ok submitted=%lld completed=%lld failed=%lld cancelled=%lld launches=%lld max_concurrent=%lld\n",
              (long long)st.submitted, (long long)st.completed, (long long)st.failed, (long long)st.cancelled,
              (long long)st.launches, (long long)st.max_concurrent_launches);
  return 0;
}
