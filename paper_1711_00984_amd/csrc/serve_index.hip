// serve_index.hip -- fills the item -> slot map of a merged serving launch.
#include "serve_index.h"

namespace dpg {

__global__ __launch_bounds__(256) void k_serve_index(ServeIndexArgs a) {
  const int64_t item = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (item >= a.item0[a.nr]) return;
  int r = 0;
  while (r + 1 < a.nr && item >= a.item0[r + 1]) ++r;
  const int64_t i = item - a.item0[r];
  const int64_t slot = a.slot0[r] + i;
  a.ids[item] = int32_t(slot);
  a.off[slot] = a.base[r] + i * a.stride;
}

hipError_t launch_serve_index(const ServeIndexArgs& a, hipStream_t st) {
  const int64_t items = a.item0[a.nr];
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_index, dim3(unsigned((items + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace dpg
