// api.cpp -- the C ABI (include/dpg.h): validation, context, single-space dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "aniso.h"
#include "condense.h"
#include "ctx.h"
#include "tables.h"
#include "terms.h"

namespace dpg {

int hip_fail(hipError_t e, const char* what) {
  return fail(DPG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int size_class(int64_t n) {
  int c = 0;
  while (n > 1) { n >>= 1; ++c; }
  return c;
}

static hipError_t launch_general(int space, int p, int prec, const GeneralArgs& a, hipStream_t st) {
  if (a.list) {
    switch (space) {
      case DPG_H1: return launch_general_list_h1(p, prec, a, st);
      case DPG_HCURL: return launch_general_list_hcurl(p, prec, a, st);
      case DPG_HDIV: return launch_general_list_hdiv(p, prec, a, st);
      case DPG_L2: return launch_general_list_l2(p, prec, a, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (space) {
    case DPG_H1: return launch_general_h1(p, prec, a, st);
    case DPG_HCURL: return launch_general_hcurl(p, prec, a, st);
    case DPG_HDIV: return launch_general_hdiv(p, prec, a, st);
    case DPG_L2: return launch_general_l2(p, prec, a, st);
    default: return hipErrorInvalidValue;
  }
}

int path_code(const dpg_geometry* geom, const dpg_opts& o) {
  const bool red = o.path == DPG_PATH_REDUCED || (o.path == DPG_PATH_AUTO && geom->kind != DPG_GEOM_TRILINEAR);
  return red ? (geom->kind == DPG_GEOM_EXTRUDED ? 2 : 1) : 0;
}

int check_common(const dpg_ctx* ctx, const dpg_geometry* geom, void* out, const dpg_opts& o) {
  if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
  if (!geom) return fail(DPG_EINVAL, "geometry is NULL");
  if (geom->kind != DPG_GEOM_TRILINEAR && geom->kind != DPG_GEOM_AFFINE && geom->kind != DPG_GEOM_EXTRUDED)
    return fail(DPG_EINVAL, "unknown geometry kind %d", geom->kind);
  if (geom->n_elem < 0) return fail(DPG_EINVAL, "negative element count");
  if (geom->n_elem > 0 && (!geom->data || !out)) return fail(DPG_EINVAL, "geometry data or output is NULL");
  if (o.prec != DPG_FP64 && o.prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", o.prec);
  if (o.path < DPG_PATH_AUTO || o.path > DPG_PATH_REDUCED) return fail(DPG_EINVAL, "unknown path %d", o.path);
  if (o.path == DPG_PATH_REDUCED && geom->kind == DPG_GEOM_TRILINEAR)
    return fail(DPG_EINVAL, "the reduced path needs affine or extruded geometry");
  if (!std::isfinite(o.w0) || !std::isfinite(o.w1)) return fail(DPG_EINVAL, "weights must be finite");
  return DPG_OK;
}

int launch_elements(const dpg_ctx* ctx, int space, int p, const dpg_geometry* geom, void* out,
                    const dpg_opts& o, const int32_t* elem_ids, int64_t n_items, const int64_t* out_offset,
                    Sched sched, hipStream_t st, const int32_t* list) {
  const int L = npoints(space, p);
  if (o.nq != 0 && o.nq != L)
    return fail(DPG_EINVAL, "nq=%d: only the default point count (%d) is built", o.nq, L);
  GeneralArgs a{};
  a.geom = geom->data;
  a.geom_kind = geom->kind;
  a.out = out;
  a.packed_len = packed_len(space, p);
  a.tab64 = ctx->d_tab64 + table_offset(L);
  a.tabR = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + table_offset(L))
                              : static_cast<const void*>(a.tab64);
  a.ftabR = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_f32) : static_cast<const void*>(ctx->d_f64);
  a.w0 = o.w0;
  a.w1 = o.w1;
  a.status = o.status;
  a.elem_ids = elem_ids;
  a.n_items = n_items;
  a.out_offset = out_offset;
  a.slab_group = sched.slab_group;
  a.diag_inline = sched.diag;
  a.list = list;
  const int pc = path_code(geom, o);
  const hipError_t e = pc == 2 ? launch_extruded(space, p, o.prec, a, st)
                     : pc == 1 ? launch_affine(space, p, o.prec, a, st)
                               : launch_general(space, p, o.prec, a, st);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return DPG_OK;
}

}  // namespace dpg

dpg_ctx::~dpg_ctx() {
  dpg::destroy_plans(this);
  if (d_tab64) (void)hipFree(d_tab64);
}

using dpg::fail;
using dpg::hip_fail;

extern "C" {

void dpg_opts_default(dpg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->prec = DPG_FP64;
  o->path = DPG_PATH_AUTO;
  o->nq = 0;
  o->w0 = 1.0;
  o->w1 = 1.0;
  o->status = nullptr;
}

const char* dpg_last_error(void) { return dpg::last_error(); }

int64_t dpg_gram_dim(int space, int p) {
  if (!dpg::valid_space(space) || p < 1 || p > DPG_P_MAX) return -1;
  return dpg::gram_dim(space, p);
}

int64_t dpg_gram_packed_len(int space, int p) {
  if (!dpg::valid_space(space) || p < 1 || p > DPG_P_MAX) return -1;
  return dpg::packed_len(space, p);
}

double dpg_general_flops(int space, int p) {
  if (!dpg::valid_space(space) || p < 1 || p > DPG_P_MAX) return -1.0;
  return dpg::general_flops(space, p);
}

double dpg_general_flops_trimmed(int space, int p) {
  if (!dpg::valid_space(space) || p < 1 || p > DPG_P_MAX) return -1.0;
  return dpg::general_flops(space, p, true);
}

int dpg_host_tables(int L, int kmax, double* zeta, double* w, double* chi, double* dchi) {
  if (L < 1 || L > 64 || kmax < 0 || kmax > dpg::KT - 1 || !zeta || !w || !chi || !dchi)
    return fail(DPG_EINVAL, "dpg_host_tables: bad arguments");
  dpg::gauss_legendre_01(L, zeta, w);
  dpg::chi_tables(L, zeta, kmax, chi, dchi);
  return DPG_OK;
}

int dpg_host_ftable(int r, int s, int kmax, double* F) {
  if (r < 0 || r > 1 || s < 0 || s > 1 || kmax < 0 || kmax > 64 || !F)
    return fail(DPG_EINVAL, "dpg_host_ftable: bad arguments");
  for (int i = 0; i <= kmax; ++i)
    for (int j = 0; j <= kmax; ++j) F[i * (kmax + 1) + j] = dpg::ftable_entry(r, s, i, j);
  return DPG_OK;
}

int dpg_tables_build(int p_max, void* stream, dpg_ctx** out) {
  if (!out) return fail(DPG_EINVAL, "ctx output pointer is NULL");
  *out = nullptr;
  if (p_max < 1 || p_max > DPG_P_MAX) return fail(DPG_EINVAL, "p_max=%d outside [1, %d]", p_max, DPG_P_MAX);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DPG_ENODEV, "no HIP device: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DPG_ENODEV, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  const int na = dpg::noalloc_init(dev);
  if (na != DPG_OK) return na;

  std::vector<double> t64(dpg::TABLE_LEN), f64(dpg::FTAB_LEN);
  std::vector<float> t32(dpg::TABLE_LEN), f32(dpg::FTAB_LEN);
  dpg::build_tables(t64.data(), t32.data(), f64.data(), f32.data());

  dpg_ctx* c = new (std::nothrow) dpg_ctx;
  if (!c) return fail(DPG_ENOMEM, "host allocation failed");
  c->p_max = p_max;
  c->device = dev;
  hipStream_t st = static_cast<hipStream_t>(stream);
  size_t bytes = dpg::TABLE_LEN * (sizeof(double) + sizeof(float)) + dpg::FTAB_LEN * (sizeof(double) + sizeof(float));
  char* base = nullptr;
  e = hipMalloc(reinterpret_cast<void**>(&base), bytes);
  if (e != hipSuccess) {
    delete c;
    return fail(DPG_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  c->d_tab64 = reinterpret_cast<double*>(base);
  c->d_f64 = c->d_tab64 + dpg::TABLE_LEN;
  c->d_tab32 = reinterpret_cast<float*>(c->d_f64 + dpg::FTAB_LEN);
  c->d_f32 = c->d_tab32 + dpg::TABLE_LEN;
  e = hipMemcpyAsync(c->d_tab64, t64.data(), dpg::TABLE_LEN * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_f64, f64.data(), dpg::FTAB_LEN * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_tab32, t32.data(), dpg::TABLE_LEN * sizeof(float), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_f32, f32.data(), dpg::FTAB_LEN * sizeof(float), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "table upload");
  }
  const int tr = dpg::load_default_tune(c);
  if (tr != DPG_OK) {
    delete c;
    return tr;
  }
  *out = c;
  return DPG_OK;
}

int dpg_ctx_destroy(dpg_ctx* ctx) {
  if (!ctx) return fail(DPG_ENOTINIT, "null context");
  delete ctx;
  return DPG_OK;
}

int dpg_gram_integrate(const dpg_ctx* ctx, int space, int p, const dpg_geometry* geom, void* out,
                       const dpg_opts* opts, void* stream) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  int rc = dpg::check_common(ctx, geom, out, o);
  if (rc) return rc;
  if (!dpg::valid_space(space)) return fail(DPG_EINVAL, "unknown space %d", space);
  if (p < 1 || p > ctx->p_max) return fail(DPG_EINVAL, "p=%d outside [1, %d]", p, ctx->p_max);
  if (o.nq != 0 && o.nq != dpg::npoints(space, p)) {
    // A rule other than the default: the quadrature path with nq points per direction, at
    // orders (p, p, p) through the routes of non-uniform orders (the uniform kernel of an
    // order whose rule has at least nq points, padded with zero-weight points, or the
    // per-direction kernel).
    if (o.path == DPG_PATH_REDUCED)
      return fail(DPG_EINVAL, "nq=%d: the reduced path integrates exactly and takes no rule", o.nq);
    if (o.nq < 1 || o.nq > dpg::ANISO_LMAX)
      return fail(DPG_EINVAL, "nq=%d outside [1, %d] (default %d)", o.nq, dpg::ANISO_LMAX, dpg::npoints(space, p));
    if (p > dpg::ANISO_PMAX)
      return fail(DPG_EINVAL, "nq=%d at p=%d: rules other than the default are supported up to p=%d", o.nq, p,
                  dpg::ANISO_PMAX);
    if (geom->n_elem == 0) return DPG_OK;
    const int32_t q[3] = {p, p, p};
    dpg_opts a = o;
    a.path = DPG_PATH_AUTO;   // GENERAL here names the quadrature path, not the per-direction kernel
    if (dpg::embed_applies(ctx, space, q, a))
      return dpg::integrate_aniso_embed(ctx, space, q, geom, out, a, static_cast<hipStream_t>(stream));
    return dpg::integrate_aniso(ctx, space, q, geom, out, o, static_cast<hipStream_t>(stream));
  }
  if (geom->n_elem == 0) return DPG_OK;
  const dpg::Sched g = dpg::tuned_sched(ctx, space, p, o.prec, dpg::path_code(geom, o), geom->n_elem);
  return dpg::launch_elements(ctx, space, p, geom, out, o, nullptr, geom->n_elem, nullptr, g,
                              static_cast<hipStream_t>(stream));
}

int dpg_adjoint_coupling(const dpg_ctx* ctx, int p, void* out, int prec, void* stream) {
  if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
  if (p < 1 || p > ctx->p_max) return fail(DPG_EINVAL, "p=%d outside [1, %d]", p, ctx->p_max);
  if (!out) return fail(DPG_EINVAL, "output is NULL");
  if (prec != DPG_FP64 && prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", prec);
  const void* F = prec == DPG_FP32 ? static_cast<const void*>(ctx->d_f32) : static_cast<const void*>(ctx->d_f64);
  const hipError_t e = dpg::launch_coupling(p, prec, F, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPG_OK : hip_fail(e, "coupling launch");
}

int dpg_replicate_blocks(const dpg_ctx* ctx, int64_t n_elem, int64_t n, int copies, const void* src, void* dst,
                         int prec, void* stream) {
  if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
  if (n_elem < 0 || n < 1) return fail(DPG_EINVAL, "n_elem=%lld, n=%lld", (long long)n_elem, (long long)n);
  if (copies < 1 || copies > 4) return fail(DPG_EINVAL, "copies=%d outside [1, 4]", copies);
  if (prec != DPG_FP64 && prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", prec);
  if (n_elem == 0) return DPG_OK;
  if (!src || !dst) return fail(DPG_EINVAL, "source or destination is NULL");
  const int64_t es = prec == DPG_FP32 ? 4 : 8, cn = n * copies;
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
  const uintptr_t s1 = s0 + uintptr_t(n_elem * (n * (n + 1) / 2) * es), d1 = d0 + uintptr_t(n_elem * (cn * (cn + 1) / 2) * es);
  if (s0 < d1 && d0 < s1) return fail(DPG_EINVAL, "source and destination overlap");
  const hipError_t e = dpg::launch_replicate(prec, src, dst, n, copies, n_elem, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPG_OK : hip_fail(e, "replicate launch");
}

int dpg_cholesky_packed(const dpg_ctx* ctx, int64_t n_elem, int64_t n, void* ap, int32_t* info, int prec,
                        void* stream) {
  if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
  if (n_elem < 0 || n < 1 || n > 16384) return fail(DPG_EINVAL, "n_elem=%lld, n=%lld", (long long)n_elem, (long long)n);
  if (prec != DPG_FP64 && prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", prec);
  if (n_elem == 0) return DPG_OK;
  if (!ap) return fail(DPG_EINVAL, "packed Grams are NULL");
  const hipError_t e = dpg::launch_potrf(prec, ap, n, n_elem, info, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPG_OK : hip_fail(e, "cholesky launch");
}

int dpg_cholesky_solve_packed(const dpg_ctx* ctx, int64_t n_elem, int64_t n, const void* up, int64_t nrhs, void* b,
                              int prec, void* stream) {
  if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
  if (n_elem < 0 || n < 1 || n > 16384) return fail(DPG_EINVAL, "n_elem=%lld, n=%lld", (long long)n_elem, (long long)n);
  if (nrhs < 1 || nrhs > (int64_t(1) << 26)) return fail(DPG_EINVAL, "nrhs=%lld", (long long)nrhs);
  if (prec != DPG_FP64 && prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", prec);
  if (n_elem == 0) return DPG_OK;
  if (!up || !b) return fail(DPG_EINVAL, "factor or right-hand side is NULL");
  const int64_t es = prec == DPG_FP32 ? 4 : 8;
  const uintptr_t u0 = reinterpret_cast<uintptr_t>(up), b0 = reinterpret_cast<uintptr_t>(b);
  const uintptr_t u1 = u0 + uintptr_t(n_elem * (n * (n + 1) / 2) * es), b1 = b0 + uintptr_t(n_elem * n * nrhs * es);
  if (u0 < b1 && b0 < u1) return fail(DPG_EINVAL, "factor and right-hand side overlap");
  const hipError_t e = dpg::launch_potrs(prec, up, n, n_elem, nrhs, b, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPG_OK : hip_fail(e, "cholesky solve launch");
}

int64_t dpg_gram_dim_aniso(int space, const int32_t* p) {
  if (!dpg::valid_space(space) || !p) return -1;
  int64_t n = 0;
  for (int d = 0; d < 3; ++d)
    if (p[d] < 1 || p[d] > dpg::ANISO_PMAX) return -1;
  for (int a = 0; a < (space == DPG_H1 || space == DPG_L2 ? 1 : 3); ++a) {
    int64_t c = 1;
    for (int d = 0; d < 3; ++d) {
      const int q = p[d];
      c *= space == DPG_H1 ? q + 1 : space == DPG_L2 ? q : space == DPG_HDIV ? (d == a ? q + 1 : q) : (d == a ? q : q + 1);
    }
    n += c;
  }
  return n;
}

static int aniso_route(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts& o) {
  if (p[0] == p[1] && p[1] == p[2] && o.nq == 0 && o.path == DPG_PATH_AUTO && p[0] <= ctx->p_max)
    return DPG_ROUTE_UNIFORM;
  return dpg::embed_applies(ctx, space, p, o) ? DPG_ROUTE_EMBEDDED : DPG_ROUTE_PER_DIRECTION;
}

int dpg_aniso_route(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts* opts) {
  if (!ctx) return fail(DPG_ENOTINIT, "context is NULL");
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  if (dpg_gram_dim_aniso(space, p) < 0) return fail(DPG_EINVAL, "invalid space or orders");
  return aniso_route(ctx, space, p, o);
}

int dpg_gram_integrate_aniso(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                             const dpg_opts* opts, void* stream) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  int rc = dpg::check_common(ctx, geom, out, o);
  if (rc) return rc;
  if (!dpg::valid_space(space)) return fail(DPG_EINVAL, "unknown space %d", space);
  if (!p) return fail(DPG_EINVAL, "orders are NULL");
  for (int d = 0; d < 3; ++d)
    if (p[d] < 1 || p[d] > dpg::ANISO_PMAX)
      return fail(DPG_EINVAL, "p[%d]=%d outside [1, %d]", d, p[d], dpg::ANISO_PMAX);
  if (o.path == DPG_PATH_REDUCED) return fail(DPG_EINVAL, "non-uniform orders use the quadrature path only");
  if (o.nq < 0 || o.nq > dpg::ANISO_LMAX) return fail(DPG_EINVAL, "nq=%d outside [0, %d]", o.nq, dpg::ANISO_LMAX);
  if (geom->n_elem == 0) return DPG_OK;
  const int route = aniso_route(ctx, space, p, o);
  if (route == DPG_ROUTE_UNIFORM) {
    // equal orders with the default rule: the uniform quadrature kernels compute the same sums
    dpg_opts u = o;
    u.path = DPG_PATH_GENERAL;
    const dpg::Sched g = dpg::tuned_sched(ctx, space, p[0], u.prec, 0, geom->n_elem);
    return dpg::launch_elements(ctx, space, p[0], geom, out, u, nullptr, geom->n_elem, nullptr, g,
                                static_cast<hipStream_t>(stream));
  }
  if (route == DPG_ROUTE_EMBEDDED)
    return dpg::integrate_aniso_embed(ctx, space, p, geom, out, o, static_cast<hipStream_t>(stream));
  return dpg::integrate_aniso(ctx, space, p, geom, out, o, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace dpg {

int integrate_aniso(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                    const dpg_opts& o, hipStream_t st) {
  dpg::AnisoArgs a{};
  a.geom = geom->data;
  a.geom_kind = geom->kind;
  a.n_elem = geom->n_elem;
  a.out = out;
  const int64_t n = dpg_gram_dim_aniso(space, p);
  a.packed_len = n * (n + 1) / 2;
  a.space = space;
  for (int d = 0; d < 3; ++d) {
    a.q[d] = p[d];
    a.L[d] = o.nq > 0 ? o.nq : (space == DPG_L2 ? p[d] : p[d] + 1);
    a.tab64[d] = ctx->d_tab64 + dpg::table_offset(a.L[d]);
    a.tabR[d] = o.prec == DPG_FP32 ? static_cast<const void*>(ctx->d_tab32 + dpg::table_offset(a.L[d]))
                                   : static_cast<const void*>(ctx->d_tab64 + dpg::table_offset(a.L[d]));
  }
  // Contraction order: the direction with the fewest points last (outermost loop; ties
  // go to the lowest direction, so uniform orders keep xi3, xi2, xi1).  Of the other two,
  // xi3 (the slowest index of the flat numbering) goes first when it is among them, which
  // lets a diagonal block skip the pairs i3 > j3.
  int dC = 0;
  for (int d = 1; d < 3; ++d)
    if (a.L[d] < a.L[dC]) dC = d;
  a.dir[0] = dC == 2 ? 1 : 2;
  a.dir[1] = 3 - dC - a.dir[0];
  a.dir[2] = dC;
  a.w0 = o.w0;
  a.w1 = o.w1;
  a.status = o.status;
  const hipError_t e = dpg::launch_aniso(o.prec, a, st);
  return e == hipSuccess ? DPG_OK : hip_fail(e, "anisotropic launch");
}

}  // namespace dpg
