// launch_limits.h -- splitting a batch of elements over several launches.
//
// One dispatch holds at most 2^32 work-items (grid size x workgroup size),
// i.e. 2^24 workgroups of 256 threads.  The element kernels launch
// n_items * ngroups workgroups (ngroups slab groups per element), so a batch
// whose count would pass the cap is split by element into consecutive
// launches of at most launch_items(ngroups) elements each.  No HIP include:
// the arithmetic is tested on the host.
#pragma once
#include <stdint.h>

namespace dpg {

constexpr int64_t MAX_WG_PER_LAUNCH = int64_t(1) << 22;

// Elements per launch for ngroups >= 1 workgroups per element (at least one).
constexpr int64_t launch_items(int ngroups) {
  return ngroups >= 1 && MAX_WG_PER_LAUNCH / ngroups >= 1 ? MAX_WG_PER_LAUNCH / ngroups : 1;
}

// Number of launches for n_items elements.
constexpr int64_t launch_count(int64_t n_items, int ngroups) {
  return n_items <= 0 ? 0 : (n_items + launch_items(ngroups) - 1) / launch_items(ngroups);
}

}  // namespace dpg
