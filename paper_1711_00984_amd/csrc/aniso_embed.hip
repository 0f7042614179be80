// aniso_embed.hip -- non-uniform orders (p1, p2, p3) on the uniform kernels.
//
// The 1D bases are hierarchical (Sections 2.4 and 2.8.2): the functions of order
// p_d in direction d are the first ones of order P = max p_d.  So the Gram of orders
// (p1, p2, p3) is a principal submatrix of the order-P Gram, provided every direction
// keeps its own rule (the text after Algorithm 2): k_embed integrates order P with
// direction d on its p_d rule, padded to order P's point count with zero-weight
// points, only over the column slabs j3 < R3(p3) the submatrix needs, and stores the
// submatrix's entries straight into the packed numbering of (p1, p2, p3) (the others
// are dropped at the store).  An explicit rule of nq points in every direction embeds
// the same way, in an order whose default rule has at least nq points.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ctx.h"
#include "kernels.h"
#include "terms.h"

namespace dpg {

namespace {

// The order of the launch: the largest p_d, raised so that its default rule has at
// least the nq points of an explicit rule.
int emb_order(int space, const int32_t* p, int nq) {
  int P = p[0];
  for (int d = 1; d < 3; ++d) P = p[d] > P ? p[d] : P;
  const int Pq = space == SP_L2 ? nq : nq - 1;
  return Pq > P ? Pq : P;
}

// Unknowns the order-P launch carries: the columns of the slabs j3 < R3(p3) of each
// component.
int64_t emb_columns(int space, const int32_t* p, int P) {
  int64_t n = 0;
  for (int b = 0; b < ncomp(space); ++b)
    n += int64_t(range1d(space, P, b, 0)) * range1d(space, P, b, 1) * range1d(space, p[2], b, 2);
  return n;
}

}  // namespace

bool embed_applies(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts& o) {
  if (o.nq < 0 || o.path != DPG_PATH_AUTO) return false;
  const int P = emb_order(space, p, o.nq);
  if (P > 10 || P > ctx->p_max) return false;
  int64_t na = 0;
  for (int a = 0; a < ncomp(space); ++a)
    na += int64_t(range1d(space, p[0], a, 0)) * range1d(space, p[1], a, 1) * range1d(space, p[2], a, 2);
  // the order-P launch computes about (columns / unknowns)^2 times the entries needed
  // (less where whole x-tiles fall outside); measured against the per-direction kernel, it
  // was faster or even up to a squared ratio of 13.8 and slower from 30 on
  const double r = double(emb_columns(space, p, P)) / double(na);
  return r * r <= 16.0;
}

int integrate_aniso_embed(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                          const dpg_opts& o, hipStream_t st) {
  const int P = emb_order(space, p, o.nq);
  const int nc = ncomp(space);
  GeneralArgs a{};
  a.geom = geom->data;
  a.geom_kind = geom->kind;
  a.n_items = geom->n_elem;
  a.item_base = 0;
  a.elem_ids = nullptr;
  a.out = out;
  a.out_offset = nullptr;
  const int L = npoints(space, P);
  a.tab64 = ctx->d_tab64 + table_offset(L);
  a.tabR = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + table_offset(L))
                              : static_cast<const void*>(ctx->d_tab64 + table_offset(L));
  for (int d = 0; d < 3; ++d) {
    const int Ld = o.nq > 0 ? o.nq : npoints(space, p[d]);
    a.emb_L[d] = Ld;
    a.emb_tab64[d] = ctx->d_tab64 + table_offset(Ld);
    a.emb_tabR[d] = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + table_offset(Ld))
                                       : static_cast<const void*>(ctx->d_tab64 + table_offset(Ld));
  }
  int64_t n = 0;
  for (int b = 0; b < 3; ++b) {
    a.emb_off[b] = int(n);
    for (int d = 0; d < 3; ++d) a.emb_R[b][d] = b < nc ? range1d(space, p[d], b, d) : 0;
    a.emb_jmax[b] = a.emb_R[b][2];
    n += int64_t(a.emb_R[b][0]) * a.emb_R[b][1] * a.emb_R[b][2];
  }
  a.emb_off[3] = int(n);
  a.packed_len = n * (n + 1) / 2;
  a.w0 = o.w0;
  a.w1 = o.w1;
  a.status = o.status;
  a.slab_group = 0;
  a.diag_inline = -1;
  a.list = nullptr;
  hipError_t e;
  switch (space) {
    case SP_H1: e = launch_embed_h1(P, o.prec, a, st); break;
    case SP_HCURL: e = launch_embed_hcurl(P, o.prec, a, st); break;
    case SP_HDIV: e = launch_embed_hdiv(P, o.prec, a, st); break;
    default: e = launch_embed_l2(P, o.prec, a, st); break;
  }
  return e == hipSuccess ? DPG_OK : hip_fail(e, "embedded non-uniform launch");
}

}  // namespace dpg
