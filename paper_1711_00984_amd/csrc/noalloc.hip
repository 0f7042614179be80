// noalloc.hip -- the uneven-batch integration without any allocation.
//
// dpg_gram_integrate_batched buckets the elements by (space, p) on the host and
// keeps each bucket's element list in device memory it allocates.  This variant
// is for callers that cannot allocate (graph capture, tight serving loops): the
// lists live in a fixed device array of this file, `scratch`, and are built on
// the device, so the host neither allocates nor waits:
//
//   1. one workgroup counts the elements of every (space, p) bucket, scans the
//      counts and scatters the element numbers into the bucket lists;
//   2. one listed launch per (space, p <= p_max) reads its bucket's count and
//      first list entry from the array; its fixed grid strides over the bucket
//      (an empty bucket's workgroups exit at once).
//
// The Gram kernels are those of the batched call, so every element's matrix is
// bit for bit the same.  The array is shared by every call on a device and keeps
// the last call's lists: two calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.h"
#include "terms.h"

namespace dpg {

constexpr int NA_PSTRIDE = DPG_P_MAX + 1;              // bucket b = space * NA_PSTRIDE + p
constexpr int NA_BUCKETS = 4 * NA_PSTRIDE;
constexpr int NA_HEADER = 128;                         // {count, first} per bucket, then padding
static_assert(2 * NA_BUCKETS <= NA_HEADER, "bucket records fit the header");
constexpr int64_t NA_MAX_ELEM = int64_t(1) << 20;      // elements per call (4 MiB of lists)
constexpr int NA_MAX_DEV = 64;
constexpr int NA_THREADS = 1024;

// The bucket records and element lists.  Its address on each device is taken
// once with hipGetSymbolAddress; host code uses only that address.
static __device__ __align__(256) int32_t scratch[NA_HEADER + NA_MAX_ELEM];

static std::mutex g_na_mu;
static int32_t* g_na_ptr[NA_MAX_DEV];

// Count, scan and scatter: the list of bucket b is scratch[NA_HEADER + first_b ..
// + count_b), its record {count_b, first_b} at scratch[2 b].  Every record is
// rewritten by every call, so nothing needs clearing beforehand.  Elements with an
// invalid space or order join no bucket; their status word says DPG_EINVAL.
__global__ void __launch_bounds__(NA_THREADS) k_na_bucket(const int8_t* __restrict__ space,
                                                         const int8_t* __restrict__ p, int64_t n, int p_max,
                                                         int32_t* __restrict__ status, int32_t* __restrict__ sc) {
  __shared__ int cnt[NA_BUCKETS], cur[NA_BUCKETS];
  const int tid = threadIdx.x;
  auto bucket = [&](int64_t e) {
    const int s = space[e], q = p[e];
    return (s >= 0 && s < 4 && q >= 1 && q <= p_max) ? s * NA_PSTRIDE + q : -1;
  };
  for (int b = tid; b < NA_BUCKETS; b += NA_THREADS) cnt[b] = 0;
  __syncthreads();
  for (int64_t e = tid; e < n; e += NA_THREADS) {
    const int b = bucket(e);
    if (b >= 0) atomicAdd(&cnt[b], 1);
    else if (status) status[e] = DPG_EINVAL;
  }
  __syncthreads();
  if (tid == 0) {
    int first = 0;
    for (int b = 0; b < NA_BUCKETS; ++b) {
      sc[2 * b] = cnt[b];
      sc[2 * b + 1] = first;
      cur[b] = first;
      first += cnt[b];
    }
  }
  __syncthreads();
  int32_t* ids = sc + NA_HEADER;
  for (int64_t e = tid; e < n; e += NA_THREADS) {
    const int b = bucket(e);
    if (b >= 0) ids[atomicAdd(&cur[b], 1)] = int32_t(e);
  }
}

// Address of the array on the current device (taken once per device).
int noalloc_init(int dev) {
  if (dev < 0 || dev >= NA_MAX_DEV) return fail(DPG_ENODEV, "device %d outside [0, %d)", dev, NA_MAX_DEV);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (g_na_ptr[dev]) return DPG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(DPG_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_na_ptr[dev] = static_cast<int32_t*>(ptr);
  return DPG_OK;
}

static int32_t* noalloc_ptr(int dev) {
  if (dev < 0 || dev >= NA_MAX_DEV) return nullptr;
  std::lock_guard<std::mutex> lk(g_na_mu);
  return g_na_ptr[dev];
}

}  // namespace dpg

using dpg::fail;
using dpg::hip_fail;

extern "C" int64_t dpg_noalloc_max_elements(void) { return dpg::NA_MAX_ELEM; }

extern "C" int dpg_gram_integrate_batched_noalloc(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                                                  const dpg_geometry* geom, const int64_t* out_offset, void* out,
                                                  const dpg_opts* opts, void* stream) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  int rc = dpg::check_common(ctx, geom, out, o);
  if (rc) return rc;
  const int64_t n = geom->n_elem;
  if (n > dpg::NA_MAX_ELEM)
    return fail(DPG_EINVAL, "%lld elements: the allocation-free batch takes at most %lld", (long long)n,
                (long long)dpg::NA_MAX_ELEM);
  if (n == 0) return DPG_OK;
  if (!space || !p || !out_offset) return fail(DPG_EINVAL, "space, p and out_offset are required");
  if (o.nq != 0) return fail(DPG_EINVAL, "batched integration uses the default point counts (nq = 0)");
  int32_t* sc = dpg::noalloc_ptr(ctx->device);
  if (!sc) return fail(DPG_ENOTINIT, "device %d has no list array (context not built on it)", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(dpg::k_na_bucket, dim3(1), dim3(dpg::NA_THREADS), 0, st, space, p, n, ctx->p_max, o.status, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bucket launch");
  // the expected bucket size sizes each listed launch's grid and slab groups
  const int64_t expect = n / (4 * ctx->p_max) + 1;
  const int pc = dpg::path_code(geom, o);
  for (int s = 0; s < 4; ++s)
    for (int q = 1; q <= ctx->p_max; ++q) {
      const int b = s * dpg::NA_PSTRIDE + q;
      const dpg::Sched g = dpg::tuned_sched(ctx, s, q, o.prec, pc, expect);
      rc = dpg::launch_elements(ctx, s, q, geom, out, o, sc + dpg::NA_HEADER, expect, out_offset, g, st, sc + 2 * b);
      if (rc != DPG_OK) return rc;
    }
  return DPG_OK;
}
