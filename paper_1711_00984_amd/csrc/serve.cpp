// serve.cpp -- the serving loop's device side (HIP streams, events, resident
// arenas) and the dpg_serve_* C ABI.
//
// Device memory of a server, reserved once at creation:
//   output arena   mem_budget_bytes, sub-allocated per admitted request
//   element slots  per slot: trilinear geometry (24 doubles), affine geometry
//                  (12 doubles), status word, output offset
//   item maps      2 * max_slots int32 (merged launches)
// plus pinned host staging of 24 doubles per slot.  Host geometry is copied
// into the staging at submit (no device work on the client's thread) and
// uploaded on the launch stream just before the request's kernels; device
// geometry is copied into the slots at submit.  A request's geometry stays in
// its slots, and its output in the arena, until release.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctx.h"
#include "serve_core.h"
#include "serve_index.h"
#include "terms.h"

namespace dpg::serve {

static_assert(kMaxMerge == SERVE_MAX_MERGE, "merge limit of the scheduler and of the item-map kernel");

namespace {

int elem_size(int prec) { return prec == DPG_FP32 ? 4 : 8; }
int geom_stride(int kind) { return kind == DPG_GEOM_AFFINE ? 12 : kind == DPG_GEOM_EXTRUDED ? 10 : 24; }

class HipExecutor final : public Executor {
 public:
  HipExecutor(const dpg_ctx* ctx, const dpg_serve_cfg& cfg) : ctx_(ctx), slots_(cfg.max_slots), n_streams_(cfg.n_streams) {}

  int init(const dpg_serve_cfg& cfg) {
    hipError_t e = hipSetDevice(ctx_->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hipMalloc(reinterpret_cast<void**>(&out_), size_t(cfg.mem_budget_bytes));
    if (e != hipSuccess)
      return fail(DPG_ENOMEM, "output arena of %lld bytes: %s", (long long)cfg.mem_budget_bytes, hipGetErrorString(e));
    const size_t per_slot = (24 + 12 + 10) * sizeof(double) + sizeof(int32_t) + sizeof(int64_t) + 2 * sizeof(int32_t);
    char* base = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&base), size_t(slots_) * per_slot);
    if (e != hipSuccess) return fail(DPG_ENOMEM, "slot arena: %s", hipGetErrorString(e));
    slot_mem_ = base;
    geo_tri_ = reinterpret_cast<double*>(base);
    geo_aff_ = geo_tri_ + 24 * slots_;
    geo_ext_ = geo_aff_ + 12 * slots_;
    off_ = reinterpret_cast<int64_t*>(geo_ext_ + 10 * slots_);
    status_ = reinterpret_cast<int32_t*>(off_ + slots_);
    ids_ = status_ + slots_;
    for (int i = 0; i < n_streams_; ++i) {
      hipStream_t s;
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
      streams_.push_back(s);
    }
    e = hipStreamCreateWithFlags(&upload_, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipHostMalloc(reinterpret_cast<void**>(&stage_), size_t(slots_) * 24 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return fail(DPG_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
    return DPG_OK;
  }

  ~HipExecutor() override {
    (void)hipSetDevice(ctx_->device);
    for (hipStream_t s : streams_) (void)hipStreamSynchronize(s);
    for (hipEvent_t ev : events_) (void)hipEventDestroy(ev);
    for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
    if (upload_) (void)hipStreamDestroy(upload_);
    if (stage_) (void)hipHostFree(stage_);
    if (slot_mem_) (void)hipFree(slot_mem_);
    if (out_) (void)hipFree(out_);
  }

  int put_geometry(const dpg_request& rq, int64_t slot0, bool* staged) override {
    const int st = geom_stride(rq.geom.kind);
    if (slot0 < 0 || slot0 + rq.geom.n_elem > slots_) return fail(DPG_EINVAL, "slot range outside the arena");
    const size_t bytes = size_t(rq.geom.n_elem) * st * sizeof(double);
    if (rq.geom_on_host) {   // slots of this request are exclusive: no copy of them is in flight
      std::memcpy(stage_ + slot0 * 24, rq.geom.data, bytes);
      *staged = true;
      return DPG_OK;
    }
    double* dst = arena(rq.geom.kind) + slot0 * st;
    std::lock_guard<std::mutex> lk(upload_mu_);
    hipError_t e = hipSetDevice(ctx_->device);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dst, rq.geom.data, bytes, hipMemcpyDeviceToDevice, upload_);
    if (e == hipSuccess) e = hipStreamSynchronize(upload_);
    return e == hipSuccess ? DPG_OK : hip_fail(e, "geometry copy");
  }

  int start(Launch& l) override {
    hipError_t e = hipSetDevice(ctx_->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = streams_.at(l.stream);
    const Work& w0 = l.work.front();
    const int es = elem_size(w0.prec);
    dpg_opts o;
    dpg_opts_default(&o);
    o.prec = w0.prec;
    o.path = w0.path;
    o.w0 = w0.w0;
    o.w1 = w0.w1;
    double* geo = arena(w0.kind);
    const int gs = geom_stride(w0.kind);
    for (const Work& w : l.work) {   // staged host geometry goes up first, in stream order
      if (!w.staged) continue;
      if (w.slot0 < 0 || w.slot0 + w.n > slots_) return fail(DPG_EINVAL, "request outside the arenas");
      e = hipMemcpyAsync(geo + w.slot0 * gs, stage_ + w.slot0 * 24, size_t(w.n) * gs * sizeof(double),
                         hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "geometry upload");
    }
    int rc = DPG_OK;
    if (w0.q[0] > 0) {
      // non-uniform orders: one call per request (its slots and output range are contiguous),
      // through the entry point's route for the orders
      for (const Work& w : l.work) {
        if (w.slot0 + w.n > slots_ || w.out_off % es) return fail(DPG_EINVAL, "request outside the arenas");
        dpg_geometry g{w.kind, 0, w.n, geo + w.slot0 * gs};
        o.status = status_ + w.slot0;
        rc = dpg_gram_integrate_aniso(ctx_, w.space, w.q, &g, out_ + w.out_off, &o, st);
        if (rc != DPG_OK) break;
      }
    } else if (l.work.size() == 1) {
      // one request: its slots and its output range are contiguous
      if (w0.slot0 + w0.n > slots_ || w0.out_off % es) return fail(DPG_EINVAL, "request outside the arenas");
      dpg_geometry g{w0.kind, 0, w0.n, geo + w0.slot0 * gs};
      o.status = status_ + w0.slot0;
      const Sched G = tuned_sched(ctx_, w0.space, w0.p, w0.prec, path_code(&g, o), w0.n);
      rc = launch_elements(ctx_, w0.space, w0.p, &g, out_ + w0.out_off, o, nullptr, w0.n, nullptr, G, st);
    } else {
      // merged: geometry, status and output offsets indexed by slot through the item map
      if (l.ids_off < 0 || l.ids_off + l.items > 2 * slots_ || int(l.work.size()) > SERVE_MAX_MERGE)
        return fail(DPG_EINVAL, "item map outside its arena");
      ServeIndexArgs a{};
      a.nr = int32_t(l.work.size());
      a.stride = w0.packed_len;
      a.ids = ids_ + l.ids_off;
      a.off = off_;
      int64_t item = 0;
      for (int r = 0; r < a.nr; ++r) {
        const Work& w = l.work[r];
        if (w.slot0 + w.n > slots_ || w.out_off % es || w.packed_len != w0.packed_len)
          return fail(DPG_EINVAL, "merged request outside the arenas");
        a.item0[r] = item;
        a.slot0[r] = w.slot0;
        a.base[r] = w.out_off / es;
        item += w.n;
      }
      a.item0[a.nr] = item;
      if (item != l.items) return fail(DPG_EINVAL, "item count mismatch");
      e = launch_serve_index(a, st);
      if (e != hipSuccess) return hip_fail(e, "item map launch");
      dpg_geometry g{w0.kind, 0, int64_t(slots_), geo};
      o.status = status_;
      const Sched G = tuned_sched(ctx_, w0.space, w0.p, w0.prec, path_code(&g, o), l.items);
      rc = launch_elements(ctx_, w0.space, w0.p, &g, out_, o, ids_ + l.ids_off, l.items, off_, G, st);
    }
    if (rc != DPG_OK) return rc;
    hipEvent_t ev;
    if (!events_free_.empty()) {
      ev = events_free_.back();
      events_free_.pop_back();
    } else {
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      events_.push_back(ev);
    }
    e = hipEventRecord(ev, st);
    if (e != hipSuccess) {
      events_free_.push_back(ev);
      return hip_fail(e, "hipEventRecord");
    }
    l.handle = ev;
    return DPG_OK;
  }

  int query(Launch& l) override {
    if (!l.handle) return 1;
    const hipError_t e = hipEventQuery(static_cast<hipEvent_t>(l.handle));
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return hip_fail(e, "launch");
  }

  void retire(Launch& l) override {
    if (l.handle) events_free_.push_back(static_cast<hipEvent_t>(l.handle));
    l.handle = nullptr;
  }

  void drain() override {
    (void)hipSetDevice(ctx_->device);
    for (hipStream_t s : streams_) (void)hipStreamSynchronize(s);
  }

  void* out_base() const override { return out_; }
  int32_t* status_base() const override { return status_; }

  int copy_out(const Work& w, int what, int64_t first, int64_t count, void* dst, void* stream) override {
    const void* src;
    size_t bytes;
    if (what == 0) {
      const size_t es = size_t(elem_size(w.prec));
      src = out_ + w.out_off + size_t(first) * size_t(w.packed_len) * es;
      bytes = size_t(count) * size_t(w.packed_len) * es;
    } else {
      src = status_ + w.slot0 + first;
      bytes = size_t(count) * sizeof(int32_t);
    }
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? DPG_OK : hip_fail(e, "result copy");
  }

 private:
  const dpg_ctx* ctx_;
  int64_t slots_;
  int n_streams_;
  char* out_ = nullptr;
  char* slot_mem_ = nullptr;
  double* geo_tri_ = nullptr;   // [slots][24] trilinear, [slots][12] affine, [slots][10] extruded
  double* geo_aff_ = nullptr;
  double* geo_ext_ = nullptr;
  double* arena(int kind) const {
    return kind == DPG_GEOM_AFFINE ? geo_aff_ : kind == DPG_GEOM_EXTRUDED ? geo_ext_ : geo_tri_;
  }
  int64_t* off_ = nullptr;
  int32_t* status_ = nullptr;
  int32_t* ids_ = nullptr;
  std::vector<hipStream_t> streams_;
  hipStream_t upload_ = nullptr;
  double* stage_ = nullptr;   // pinned, 24 doubles per slot
  std::mutex upload_mu_;
  std::vector<hipEvent_t> events_, events_free_;   // events_free_ is used under the server lock
};

}  // namespace
}  // namespace dpg::serve

struct dpg_server {
  std::unique_ptr<dpg::serve::Server> s;
};

using dpg::fail;

extern "C" {

void dpg_serve_cfg_default(dpg_serve_cfg* c) {
  if (!c) return;
  *c = dpg_serve_cfg{};
  c->mem_budget_bytes = int64_t(1) << 30;
  c->max_slots = int64_t(1) << 18;
  c->max_inflight = 64;
  c->max_queue = 4096;
  c->n_streams = 4;
  c->max_merge = 32;
  c->test_executor = 0;
  c->test_fail_launch = 0;
  c->test_bytes_per_s = 1e12;
  c->test_launch_s = 0.0;
}

int dpg_serve_create(dpg_ctx* ctx, const dpg_serve_cfg* cfg, dpg_server** srv) {
  if (!srv) return fail(DPG_EINVAL, "server output pointer is NULL");
  *srv = nullptr;
  dpg_serve_cfg c;
  if (cfg) c = *cfg; else dpg_serve_cfg_default(&c);
  int rc = dpg::serve::check_cfg(c);
  if (rc) return rc;
  try {
    std::unique_ptr<dpg::serve::Executor> ex;
    int p_max = DPG_P_MAX;
    if (c.test_executor == 1) {
      if (ctx) p_max = ctx->p_max;
      ex = dpg::serve::make_stub_executor(c);
    } else {
      if (!ctx || !ctx->d_tab64) return fail(DPG_ENOTINIT, "null or destroyed context");
      p_max = ctx->p_max;
      auto h = std::make_unique<dpg::serve::HipExecutor>(ctx, c);
      rc = h->init(c);
      if (rc) return rc;
      ex = std::move(h);
    }
    auto* s = new dpg_server;
    s->s = std::make_unique<dpg::serve::Server>(c, p_max, std::move(ex));
    *srv = s;
  } catch (const std::bad_alloc&) {
    return fail(DPG_ENOMEM, "host allocation failed");
  } catch (const std::exception& x) {
    return fail(DPG_ENOMEM, "server start failed: %s", x.what());
  }
  return DPG_OK;
}

int dpg_serve_submit(dpg_server* srv, const dpg_request* req, uint64_t* ticket) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  if (!req) return fail(DPG_EINVAL, "request is NULL");
  return srv->s->submit(*req, ticket);
}

int dpg_serve_submit_chunked(dpg_server* srv, const dpg_request* req, int64_t max_chunk_bytes, uint64_t* first_ticket,
                             int64_t* n_chunks, int64_t* chunk_elems) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  if (!req) return fail(DPG_EINVAL, "request is NULL");
  return srv->s->submit_chunked(*req, max_chunk_bytes, first_ticket, n_chunks, chunk_elems);
}

int dpg_serve_poll(dpg_server* srv, uint64_t ticket, dpg_result* res) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  return srv->s->poll(ticket, res);
}

int dpg_serve_read(dpg_server* srv, uint64_t ticket, void* dst, int64_t first, int64_t count, void* stream) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  return srv->s->read(ticket, 0, dst, first, count, stream);
}

int dpg_serve_read_status(dpg_server* srv, uint64_t ticket, int32_t* dst, int64_t first, int64_t count,
                          void* stream) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  return srv->s->read(ticket, 1, dst, first, count, stream);
}

int dpg_serve_release(dpg_server* srv, uint64_t ticket) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  return srv->s->release(ticket);
}

int dpg_serve_stats_get(dpg_server* srv, dpg_serve_stats* st) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  if (!st) return fail(DPG_EINVAL, "stats pointer is NULL");
  srv->s->stats(st);
  return DPG_OK;
}

int dpg_serve_stats_reset(dpg_server* srv) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  srv->s->reset_stats();
  return DPG_OK;
}

int dpg_serve_destroy(dpg_server* srv) {
  if (!srv) return fail(DPG_ENOTINIT, "null server");
  delete srv;
  return DPG_OK;
}

}  // extern "C"
