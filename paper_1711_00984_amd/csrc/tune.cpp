// tune.cpp -- autotuner for the work decomposition of the integration kernels.
//
// The tunables are the number of column slabs one workgroup integrates (1 ..
// all slabs of an element) and, on the general path, where the diagonal
// (i3 = j3) pairs of the diagonal blocks go.  More slabs per workgroup
// amortise the metric evaluation and the per-block table registers over more
// pairs; fewer give more, smaller workgroups (load balance, occupancy of the
// tail).  A diagonal pair that closes its slab in the full x tiling costs
// extra MFMA work on its lower triangle but writes the line it shares with
// the slab's last off-diagonal segment right after it, so the L2 merges the
// two halves instead of writing them back to HBM separately.  The best
// choice depends on (space, p, precision, path) and on the batch size, so
// the tuner times the candidates on the caller's data and records the
// winner per batch-size class (floor(log2(n_elem))).  The table can be saved
// to and loaded from a small JSON file keyed by the GPU architecture.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "terms.h"

namespace dpg {

static int nslab(int space, int p) {
  int o = 0;
  for (int b = 0; b < ncomp(space); ++b) o += range1d(space, p, b, 2);
  return o;
}

Sched tuned_sched(const dpg_ctx* ctx, int space, int p, int prec, int path, int64_t n) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  dpg::Sched best;
  if (ctx->tune.empty()) return best;
  const int sc = size_class(n);
  int bestd = 3;
  for (const auto& kv : ctx->tune) {
    const TuneKey& k = kv.first;
    if (k.space != space || k.p != p || k.prec != prec || k.reduced != path) continue;
    const int d = std::abs(k.size_class - sc);
    if (d < bestd) { bestd = d; best = Sched{kv.second.slab_group, kv.second.diag}; }
  }
  return best;
}

// The tuning table shipped with the library: DPG_TUNE_TABLE names a file (an empty
// value: none), else tune_gfx950.json next to libdpg.so.  A missing file leaves the
// heuristic defaults.
int load_default_tune(dpg_ctx* ctx) {
  const char* env = std::getenv("DPG_TUNE_TABLE");
  std::string path;
  if (env) {
    if (!*env) return DPG_OK;
    path = env;
  } else {
    Dl_info info;
    if (!dladdr(reinterpret_cast<void*>(&dpg_tune_load), &info) || !info.dli_fname) return DPG_OK;
    path = info.dli_fname;
    const size_t slash = path.rfind('/');
    path = (slash == std::string::npos ? std::string() : path.substr(0, slash + 1)) + "tune_gfx950.json";
  }
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return env ? fail(DPG_EINVAL, "DPG_TUNE_TABLE=%s: cannot read", path.c_str()) : DPG_OK;
  std::fclose(f);
  return dpg_tune_load(ctx, path.c_str());
}

}  // namespace dpg

using dpg::fail;
using dpg::hip_fail;

extern "C" {

int dpg_tune_clear(dpg_ctx* ctx) {
  if (!ctx) return fail(DPG_ENOTINIT, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tune.clear();
  return DPG_OK;
}

int dpg_autotune(dpg_ctx* ctx, int space, int p, const dpg_geometry* geom, void* out, const dpg_opts* opts,
                 void* stream, int* slab_group) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  int rc = dpg::check_common(ctx, geom, out, o);
  if (rc) return rc;
  if (!dpg::valid_space(space)) return fail(DPG_EINVAL, "unknown space %d", space);
  if (p < 1 || p > ctx->p_max) return fail(DPG_EINVAL, "p=%d outside [1, %d]", p, ctx->p_max);
  const int64_t n = geom->n_elem;
  if (n == 0) {
    if (slab_group) *slab_group = 0;
    return DPG_OK;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int ns = dpg::nslab(space, p);
  std::vector<int> cand;
  for (int g = 1; g < ns; g *= 2) cand.push_back(g);
  for (int g : {3, 6, 12}) if (g < ns) cand.push_back(g);
  cand.push_back(ns);
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipEvent_t e0, e1;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
  const int red = dpg::path_code(geom, o);
  std::vector<int> diags = {-1};
  if (!red) diags = dpg::diag_inline_ok(space, p) ? std::vector<int>{0, 1} : std::vector<int>{0};
  dpg::Sched best;
  float best_ms = 1e30f;
  for (int g : cand)
  for (int dg : diags) {
    float t = 1e30f;
    for (int rep = 0; rep < 4 && rc == DPG_OK; ++rep) {
      he = hipEventRecord(e0, st);
      if (he != hipSuccess) { rc = hip_fail(he, "hipEventRecord"); break; }
      rc = dpg::launch_elements(ctx, space, p, geom, out, o, nullptr, n, nullptr, dpg::Sched{g, dg}, st);
      if (rc) break;
      he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) { rc = hip_fail(he, "timing"); break; }
      if (rep > 0) t = std::min(t, ms);   // the first run warms up
    }
    if (rc) break;
    if (t < best_ms) { best_ms = t; best = dpg::Sched{g, dg}; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tune[dpg::TuneKey{space, p, o.prec, red, dpg::size_class(n)}] = dpg::TuneVal{best.slab_group, best_ms, best.diag};
  }
  if (slab_group) *slab_group = best.slab_group;
  return DPG_OK;
}

int dpg_tune_save(const dpg_ctx* ctx, const char* path) {
  if (!ctx) return fail(DPG_ENOTINIT, "null context");
  if (!path) return fail(DPG_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(DPG_EINVAL, "cannot write %s", path);
  std::lock_guard<std::mutex> lk(ctx->mu);
  std::fprintf(f, "{\"arch\": \"gfx950\", \"fields\": [\"space\", \"p\", \"prec\", \"reduced\", \"size_class\", "
                  "\"slab_group\", \"ms\", \"diag\"],\n \"tune\": [");
  bool first = true;
  for (const auto& kv : ctx->tune) {
    const auto& k = kv.first;
    std::fprintf(f, "%s\n  [%d, %d, %d, %d, %d, %d, %.6g, %d]", first ? "" : ",", k.space, k.p, k.prec, k.reduced,
                 k.size_class, kv.second.slab_group, double(kv.second.ms), kv.second.diag);
    first = false;
  }
  std::fprintf(f, "\n ]}\n");
  std::fclose(f);
  return DPG_OK;
}

int dpg_tune_load(dpg_ctx* ctx, const char* path) {
  if (!ctx) return fail(DPG_ENOTINIT, "null context");
  if (!path) return fail(DPG_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(DPG_EINVAL, "cannot read %s", path);
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
  std::fclose(f);
  if (s.find("\"gfx950\"") == std::string::npos) return fail(DPG_EINVAL, "%s: not a gfx950 tuning table", path);
  const size_t t = s.find("\"tune\"");
  if (t == std::string::npos) return fail(DPG_EINVAL, "%s: no \"tune\" array", path);
  std::vector<std::pair<dpg::TuneKey, dpg::TuneVal>> rows;
  size_t pos = s.find('[', t);
  if (pos == std::string::npos) return fail(DPG_EINVAL, "%s: malformed", path);
  ++pos;
  while (true) {
    const size_t a = s.find('[', pos);
    const size_t close = s.find(']', pos);
    if (a == std::string::npos || (close != std::string::npos && close < a)) break;
    int v[6], diag = -1;
    double ms;
    // rows without the diagonal schedule (older tables) keep its default
    const int got = std::sscanf(s.c_str() + a + 1, " %d , %d , %d , %d , %d , %d , %lf , %d", &v[0], &v[1], &v[2],
                                &v[3], &v[4], &v[5], &ms, &diag);
    if (got != 7 && got != 8) return fail(DPG_EINVAL, "%s: malformed row", path);
    if (!dpg::valid_space(v[0]) || v[1] < 1 || v[1] > DPG_P_MAX || v[5] < 1 || diag < -1 || diag > 1)
      return fail(DPG_EINVAL, "%s: invalid row", path);
    rows.push_back({dpg::TuneKey{v[0], v[1], v[2], v[3], v[4]}, dpg::TuneVal{v[5], float(ms), diag}});
    pos = s.find(']', a);
    if (pos == std::string::npos) break;
    ++pos;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (const auto& r : rows) ctx->tune[r.first] = r.second;
  return DPG_OK;
}

int dpg_tune_lookup(const dpg_ctx* ctx, int space, int p, int prec, int reduced, int64_t n_elem) {
  if (!ctx || !dpg::valid_space(space)) return -1;
  return dpg::tuned_sched(ctx, space, p, prec, reduced, n_elem).slab_group;
}

}  // extern "C"
