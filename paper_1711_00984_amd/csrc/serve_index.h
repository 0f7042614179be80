// serve_index.h -- item -> slot map of a merged serving launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpg {

constexpr int SERVE_MAX_MERGE = 32;

// Requests r = 0..nr-1 of one launch occupy element slots
// [slot0[r], slot0[r] + item0[r+1] - item0[r]) and output entries starting at
// base[r] (in elements of the output type), stride entries per element.  The
// kernel writes ids[item] = slot of the item and off[slot] = output offset of
// the element in that slot; the Gram kernels then index geometry, status and
// output by slot.
struct ServeIndexArgs {
  int32_t nr;
  int32_t reserved;
  int64_t stride;
  int32_t* ids;                         // [item0[nr]]
  int64_t* off;                         // slot-indexed
  int64_t item0[SERVE_MAX_MERGE + 1];
  int64_t slot0[SERVE_MAX_MERGE];
  int64_t base[SERVE_MAX_MERGE];
};

hipError_t launch_serve_index(const ServeIndexArgs& a, hipStream_t st);

}  // namespace dpg
