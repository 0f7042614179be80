// batch.cpp -- uneven-order batches: plan once, replay a captured HIP graph.
//
// A batch mixes spaces and orders; every (space, p) needs its own kernel
// instance (register, LDS and tile shapes are compile-time).  The planner
// reads the per-element (space, p) arrays once, buckets the elements with a
// counting sort, uploads the bucket index lists, and captures one kernel
// launch per bucket into a child graph.  The child graphs are independent
// nodes of one parent graph, so the buckets run concurrently on the device
// and the tail of one bucket overlaps the others.  The instantiated graph is
// cached per context, keyed by the call's pointers, sizes, options and a hash
// of the (space, p) contents; a repeated identical batch only re-reads the
// (space, p) arrays and replays the graph on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "ctx.h"
#include "terms.h"

namespace dpg {

struct BatchPlan {
  const void* space = nullptr;
  const void* p = nullptr;
  const void* geom = nullptr;
  int geom_kind = 0;
  int64_t n = 0;
  const void* off = nullptr;
  void* out = nullptr;
  int prec = 0, path = 0;
  double w0 = 0, w1 = 0;
  void* status = nullptr;
  uint64_t hash = 0;
  int32_t* d_ids = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;   // recorded after every replay
  int nbuckets = 0;
  ~BatchPlan() {
    // Replays of one executable graph run in launch order, so the last replay's event
    // covers them all; only this plan's work is waited for, not the device.
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_ids) (void)hipFree(d_ids);
  }
};

void destroy_plans(dpg_ctx* c) {
  std::lock_guard<std::mutex> lk(c->mu);
  c->plans.clear();
}

static uint64_t fnv1a(const int8_t* a, const int8_t* b, int64_t n) {
  uint64_t h = 1469598103934665603ull;
  for (int64_t i = 0; i < n; ++i) {
    h = (h ^ uint8_t(a[i])) * 1099511628211ull;
    h = (h ^ uint8_t(b[i])) * 1099511628211ull;
  }
  return h;
}

constexpr int kMaxPlans = 8;

}  // namespace dpg

using dpg::fail;
using dpg::hip_fail;

namespace dpg {

// Plan (or find the cached plan of) the batch whose per-element space and order are
// hs, hp (host copies) and replay it on st.  key_space, key_p: the caller's arrays,
// part of the plan's key with the contents' hash.
static int batched_run(const dpg_ctx* ctx, const int8_t* hs, const int8_t* hp, const void* space, const void* p,
                       const dpg_geometry* geom, const int64_t* out_offset, void* out, const dpg_opts& o,
                       hipStream_t st) {
  const int64_t n = geom->n_elem;
  int rc = DPG_OK;
  hipError_t e = hipSuccess;
  for (int64_t i = 0; i < n; ++i)
    if (!dpg::valid_space(hs[i]) || hp[i] < 1 || hp[i] > ctx->p_max)
      return fail(DPG_EINVAL, "element %lld: space=%d p=%d invalid", (long long)i, hs[i], hp[i]);
  const uint64_t h = dpg::fnv1a(hs, hp, n);

  std::shared_ptr<dpg::BatchPlan> plan;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (size_t i = 0; i < ctx->plans.size(); ++i) {
      const auto& q = ctx->plans[i];
      if (q->space == space && q->p == p && q->geom == geom->data && q->geom_kind == geom->kind && q->n == n &&
          q->off == out_offset && q->out == out && q->prec == o.prec && q->path == o.path && q->w0 == o.w0 &&
          q->w1 == o.w1 && q->status == o.status && q->hash == h) {
        plan = q;
        ctx->plans.erase(ctx->plans.begin() + i);
        ctx->plans.push_back(plan);   // most recently used last
        break;
      }
    }
  }
  if (!plan) {
    // ---- plan: counting sort by (space, p), heaviest buckets first
    const int NB = 4 * (DPG_P_MAX + 1);
    std::vector<int64_t> cnt(NB + 1, 0);
    for (int64_t i = 0; i < n; ++i) cnt[hs[i] * (DPG_P_MAX + 1) + hp[i] + 1]++;
    for (int b = 0; b < NB; ++b) cnt[b + 1] += cnt[b];
    std::vector<int32_t> ids(n);
    {
      std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
      for (int64_t i = 0; i < n; ++i) ids[pos[hs[i] * (DPG_P_MAX + 1) + hp[i]]++] = int32_t(i);
    }
    std::vector<int> order;
    for (int b = 0; b < NB; ++b)
      if (cnt[b + 1] > cnt[b]) order.push_back(b);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const int sx = x / (DPG_P_MAX + 1), px = x % (DPG_P_MAX + 1);
      const int sy = y / (DPG_P_MAX + 1), py = y % (DPG_P_MAX + 1);
      return dpg::packed_len(sx, px) * (cnt[x + 1] - cnt[x]) > dpg::packed_len(sy, py) * (cnt[y + 1] - cnt[y]);
    });
    auto q = std::make_shared<dpg::BatchPlan>();
    q->space = space; q->p = p; q->geom = geom->data; q->geom_kind = geom->kind; q->n = n;
    q->off = out_offset; q->out = out; q->prec = o.prec; q->path = o.path; q->w0 = o.w0; q->w1 = o.w1;
    q->status = o.status; q->hash = h; q->nbuckets = int(order.size());
    e = hipMalloc(reinterpret_cast<void**>(&q->d_ids), n * sizeof(int32_t));
    if (e != hipSuccess) return fail(DPG_ENOMEM, "hipMalloc ids: %s", hipGetErrorString(e));
    e = hipMemcpy(q->d_ids, ids.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload ids");
    // ---- capture one child graph per bucket, all independent in the parent
    hipStream_t side;
    e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipGraphCreate(&q->graph, 0);
    for (size_t k = 0; k < order.size() && e == hipSuccess && rc == DPG_OK; ++k) {
      const int b = order[k];
      const int sp = b / (DPG_P_MAX + 1), pp = b % (DPG_P_MAX + 1);
      const int64_t m = cnt[b + 1] - cnt[b];
      const dpg::Sched g = dpg::tuned_sched(ctx, sp, pp, o.prec, dpg::path_code(geom, o), m);
      e = hipStreamBeginCapture(side, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) break;
      rc = dpg::launch_elements(ctx, sp, pp, geom, out, o, q->d_ids + cnt[b], m, out_offset, g, side);
      hipGraph_t child = nullptr;
      const hipError_t e2 = hipStreamEndCapture(side, &child);
      if (rc != DPG_OK) { if (child) (void)hipGraphDestroy(child); break; }
      e = e2;
      if (e != hipSuccess) break;
      hipGraphNode_t node;
      e = hipGraphAddChildGraphNode(&node, q->graph, nullptr, 0, child);
      (void)hipGraphDestroy(child);
    }
    (void)hipStreamDestroy(side);
    if (rc != DPG_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    e = hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    e = hipEventCreateWithFlags(&q->done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    plan = q;
    std::vector<std::shared_ptr<dpg::BatchPlan>> evicted;   // destroyed after the lock is released
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->plans.push_back(q);
    while (int(ctx->plans.size()) > dpg::kMaxPlans) {
      evicted.push_back(ctx->plans.front());
      ctx->plans.erase(ctx->plans.begin());
    }
  }
  e = hipGraphLaunch(plan->exec, st);
  if (e == hipSuccess) e = hipEventRecord(plan->done, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return DPG_OK;
}

static int batched_check(const dpg_ctx* ctx, const int8_t* space, const int8_t* p, const dpg_geometry* geom,
                         const int64_t* out_offset, void* out, const dpg_opts& o) {
  int rc = dpg::check_common(ctx, geom, out, o);
  if (rc) return rc;
  const int64_t n = geom->n_elem;
  if (n > 0 && (!space || !p || !out_offset)) return fail(DPG_EINVAL, "space, p and out_offset are required");
  if (n > int64_t(0x7fffffff)) return fail(DPG_EINVAL, "batch too large (%lld elements)", (long long)n);
  if (o.nq != 0) return fail(DPG_EINVAL, "batched integration uses the default point counts (nq = 0)");
  return DPG_OK;
}

}  // namespace dpg

extern "C" int dpg_gram_integrate_batched(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                                          const dpg_geometry* geom, const int64_t* out_offset, void* out,
                                          const dpg_opts* opts, void* stream) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  const int rc = dpg::batched_check(ctx, space, p, geom, out_offset, out, o);
  if (rc || geom->n_elem == 0) return rc;
  const int64_t n = geom->n_elem;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int8_t> hs(n), hp(n);
  hipError_t e = hipMemcpyAsync(hs.data(), space, n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), p, n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "reading space/p");
  return dpg::batched_run(ctx, hs.data(), hp.data(), space, p, geom, out_offset, out, o, st);
}

extern "C" int dpg_gram_integrate_batched_host(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                                               const dpg_geometry* geom, const int64_t* out_offset, void* out,
                                               const dpg_opts* opts, void* stream) {
  dpg_opts o;
  if (opts) o = *opts; else dpg_opts_default(&o);
  const int rc = dpg::batched_check(ctx, space, p, geom, out_offset, out, o);
  if (rc || geom->n_elem == 0) return rc;
  return dpg::batched_run(ctx, space, p, space, p, geom, out_offset, out, o, static_cast<hipStream_t>(stream));
}

extern "C" int dpg_batch_plans(const dpg_ctx* ctx) {
  if (!ctx) return -1;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return int(ctx->plans.size());
}
