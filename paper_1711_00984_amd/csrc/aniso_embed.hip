// aniso_embed.hip -- non-uniform orders (p1, p2, p3) on the uniform kernels.
//
// The 1D bases are hierarchical (Sections 2.4 and 2.8.2): the functions of order
// p_d in direction d are the first ones of order P = max p_d.  So the Gram of orders
// (p1, p2, p3) is a principal submatrix of the order-P Gram, provided every direction
// keeps its own rule (the text after Algorithm 2): k_embed integrates order P with
// direction d on its p_d rule, padded to order P's point count with zero-weight
// points, and only over the column slabs j3 < R3(p3) the submatrix needs.  Its
// order-P packed output goes to a scratch buffer, and k_embed_gather copies the
// submatrix into the packed numbering of (p1, p2, p3).
//
// The scratch comes from a stream-ordered pool of the context that keeps its memory
// between calls (at most EMB_SCRATCH bytes per call; larger batches run in chunks).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ctx.h"
#include "kernels.h"
#include "metric.h"
#include "terms.h"

namespace dpg {

constexpr int EMB_DIM_MAX = 4096;                          // 3 * 10 * 11 * 11 = 3630 at orders <= 10
constexpr int64_t EMB_SCRATCH = int64_t(4) << 30;           // scratch bytes per call
constexpr int64_t EMB_SLICE = 4096;                         // packed entries per gather item
constexpr int EMB_GRID = 4096;

// Submatrix numbering: component a of orders (p1, p2, p3) spans ra[a][d] functions in
// direction d from offset offa[a]; order P's spans ru[a][d] from offu[a].
struct EmbedMap {
  int nc;
  int ra[3][3], ru[3][3];
  int offa[4], offu[4];
  int64_t plen_a, plen_u;
};

template <typename Real>
__global__ void __launch_bounds__(256) k_embed_gather(const Real* __restrict__ src, Real* __restrict__ dst,
                                                      int64_t n_elem, int64_t slices, EmbedMap m) {
  __shared__ int s_map[EMB_DIM_MAX];   // submatrix index -> order-P index
  const int n = m.offa[m.nc];
  for (int i = threadIdx.x; i < n; i += 256) {
    int a = 0;
    while (a + 1 < m.nc && i >= m.offa[a + 1]) ++a;
    int r = i - m.offa[a];
    const int i1 = r % m.ra[a][0];
    r /= m.ra[a][0];
    const int i2 = r % m.ra[a][1], i3 = r / m.ra[a][1];
    s_map[i] = m.offu[a] + i1 + m.ru[a][0] * (i2 + m.ru[a][1] * i3);
  }
  __syncthreads();
  for (int64_t item = blockIdx.x; item < n_elem * slices; item += gridDim.x) {
    const int64_t e = item / slices, k0 = (item % slices) * EMB_SLICE;
    const int64_t k1 = k0 + EMB_SLICE < m.plen_a ? k0 + EMB_SLICE : m.plen_a;
    const Real* se = src + e * m.plen_u;
    Real* de = dst + e * m.plen_a;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
      // packed 'U' entry k = I + J (J + 1) / 2, I <= J
      int64_t J = int64_t((sqrt(8.0 * double(k) + 1.0) - 1.0) * 0.5);
      while (J * (J + 1) / 2 > k) --J;
      while ((J + 1) * (J + 2) / 2 <= k) ++J;
      const int I = int(k - J * (J + 1) / 2);
      const int64_t uJ = s_map[J];
      de[k] = se[int64_t(s_map[I]) + uJ * (uJ + 1) / 2];
    }
  }
}

namespace {

int emb_order(const int32_t* p) {
  int P = p[0];
  for (int d = 1; d < 3; ++d) P = p[d] > P ? p[d] : P;
  return P;
}

// Unknowns the order-P launch carries: the columns of the slabs j3 < R3(p3) of each
// component.
int64_t emb_columns(int space, const int32_t* p) {
  const int P = emb_order(p);
  int64_t n = 0;
  for (int b = 0; b < ncomp(space); ++b)
    n += int64_t(range1d(space, P, b, 0)) * range1d(space, P, b, 1) * range1d(space, p[2], b, 2);
  return n;
}

hipError_t launch_embed(int space, int p, int prec, const GeneralArgs& a, hipStream_t st) {
  switch (space) {
    case SP_H1: return launch_embed_h1(p, prec, a, st);
    case SP_HCURL: return launch_embed_hcurl(p, prec, a, st);
    case SP_HDIV: return launch_embed_hdiv(p, prec, a, st);
    default: return launch_embed_l2(p, prec, a, st);
  }
}

}  // namespace

bool embed_applies(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts& o) {
  if (o.nq != 0 || o.path != DPG_PATH_AUTO) return false;
  const int P = emb_order(p);
  if (P > 10 || P > ctx->p_max) return false;
  int64_t na = 0;
  for (int a = 0; a < ncomp(space); ++a)
    na += int64_t(range1d(space, p[0], a, 0)) * range1d(space, p[1], a, 1) * range1d(space, p[2], a, 2);
  // the order-P launch computes about (columns / unknowns)^2 times the entries needed;
  // the uniform kernels run the same sums 5-8x faster than the per-direction kernel
  const double r = double(emb_columns(space, p)) / double(na);
  return r * r <= 4.0;
}

int integrate_aniso_embed(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                          const dpg_opts& o, hipStream_t st) {
  const int P = emb_order(p);
  const int nc = ncomp(space);
  const int64_t sz = o.prec == DPG_FP32 ? 4 : 8;
  EmbedMap m{};
  m.nc = nc;
  for (int a = 0; a <= nc; ++a) {
    m.offa[a] = a == 0 ? 0 : m.offa[a - 1] + m.ra[a - 1][0] * m.ra[a - 1][1] * m.ra[a - 1][2];
    m.offu[a] = comp_off(space, P, a);
    if (a < nc)
      for (int d = 0; d < 3; ++d) {
        m.ra[a][d] = range1d(space, p[d], a, d);
        m.ru[a][d] = range1d(space, P, a, d);
      }
  }
  const int64_t na = m.offa[nc];
  m.plen_a = na * (na + 1) / 2;
  m.plen_u = packed_len(space, P);

  GeneralArgs a{};
  a.geom_kind = geom->kind;
  a.elem_ids = nullptr;
  a.out_offset = nullptr;
  a.packed_len = m.plen_u;
  const int L = npoints(space, P);
  a.tab64 = ctx->d_tab64 + table_offset(L);
  a.tabR = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + table_offset(L))
                              : static_cast<const void*>(ctx->d_tab64 + table_offset(L));
  for (int d = 0; d < 3; ++d) {
    const int Ld = npoints(space, p[d]);
    a.emb_L[d] = Ld;
    a.emb_tab64[d] = ctx->d_tab64 + table_offset(Ld);
    a.emb_tabR[d] = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + table_offset(Ld))
                                       : static_cast<const void*>(ctx->d_tab64 + table_offset(Ld));
  }
  for (int b = 0; b < 3; ++b) a.emb_jmax[b] = b < nc ? range1d(space, p[2], b, 2) : 0;
  a.w0 = o.w0;
  a.w1 = o.w1;
  a.slab_group = 0;
  a.diag_inline = -1;
  a.list = nullptr;

  const int64_t E = geom->n_elem;
  const int64_t per = m.plen_u * sz;
  int64_t chunk = EMB_SCRATCH / per;
  if (chunk < 1) chunk = 1;
  if (chunk > E) chunk = E;
  void* scratch = nullptr;
  hipError_t e = hipMallocFromPoolAsync(&scratch, size_t(chunk * per), ctx_scratch_pool(ctx), st);
  if (e != hipSuccess) return hip_fail(e, "scratch allocation of the embedded launch");
  const int ng = geom_stride(geom->kind);
  const int64_t slices = (m.plen_a + EMB_SLICE - 1) / EMB_SLICE;
  for (int64_t c0 = 0; c0 < E && e == hipSuccess; c0 += chunk) {
    const int64_t n = E - c0 < chunk ? E - c0 : chunk;
    a.geom = geom->data + c0 * ng;
    a.status = o.status ? o.status + c0 : nullptr;
    a.n_items = n;
    a.item_base = 0;
    a.out = scratch;
    e = launch_embed(space, P, o.prec, a, st);
    if (e != hipSuccess) break;
    const unsigned grid = unsigned(n * slices < EMB_GRID ? n * slices : EMB_GRID);
    if (o.prec == DPG_FP32)
      hipLaunchKernelGGL(k_embed_gather<float>, dim3(grid), dim3(256), 0, st, static_cast<const float*>(scratch),
                         static_cast<float*>(out) + c0 * m.plen_a, n, slices, m);
    else
      hipLaunchKernelGGL(k_embed_gather<double>, dim3(grid), dim3(256), 0, st, static_cast<const double*>(scratch),
                         static_cast<double*>(out) + c0 * m.plen_a, n, slices, m);
    e = hipGetLastError();
  }
  const hipError_t ef = hipFreeAsync(scratch, st);
  if (e == hipSuccess) e = ef;
  return e == hipSuccess ? DPG_OK : hip_fail(e, "embedded non-uniform launch");
}

}  // namespace dpg
