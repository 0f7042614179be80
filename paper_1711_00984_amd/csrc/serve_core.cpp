// serve_core.cpp -- scheduler of the serving loop (host only, no HIP).
#include "serve_core.h"

#include <algorithm>
#include <cmath>
#include <tuple>

#include "errors.h"
#include "terms.h"

namespace dpg::serve {

// ---------------------------------------------------------------- RangeAlloc

RangeAlloc::RangeAlloc(int64_t capacity, int64_t align) : align_(align > 0 ? align : 1) {
  cap_ = capacity / align_ * align_;
  if (cap_ > 0) free_[0] = cap_;
}

int64_t RangeAlloc::alloc(int64_t n) {
  n = round(n);
  if (n <= 0) return -1;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < n) continue;
    const int64_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > n) free_[off + n] = len - n;
    used_ += n;
    return off;
  }
  return -1;
}

void RangeAlloc::release(int64_t off, int64_t n) {
  n = round(n);
  if (n <= 0) return;
  used_ -= n;
  auto it = free_.emplace(off, n).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {   // merge with the next range
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {                                          // and with the previous one
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

// ---------------------------------------------------------------- Server

namespace {

int elem_bytes(int prec) { return prec == DPG_FP32 ? 4 : 8; }

bool same_key(const Work& a, const Work& b) {
  return a.space == b.space && a.p == b.p && a.prec == b.prec && a.path == b.path && a.kind == b.kind &&
         a.w0 == b.w0 && a.w1 == b.w1 && a.q[0] == b.q[0] && a.q[1] == b.q[1] && a.q[2] == b.q[2];
}

// nearest-rank percentile of an unsorted sample (copied)
double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  size_t k = size_t(std::ceil(q * double(v.size())));
  k = std::clamp<size_t>(k, 1, v.size()) - 1;
  std::nth_element(v.begin(), v.begin() + k, v.end());
  return v[k];
}

}  // namespace

Server::Server(const dpg_serve_cfg& cfg, int p_max, std::unique_ptr<Executor> ex)
    : cfg_(cfg),
      p_max_(p_max),
      ex_(std::move(ex)),
      out_alloc_(cfg.mem_budget_bytes, 256),
      slot_alloc_(cfg.max_slots, 1),
      ids_alloc_(2 * cfg.max_slots, 64),
      t0_(std::chrono::steady_clock::now()) {
  thr_ = std::thread([this] { loop(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  thr_.join();
  ex_->drain();
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& [id, l] : launches_) ex_->retire(l);
  launches_.clear();
}

double Server::now() const {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
}

int Server::prepare(const dpg_request& rq, Req& r, double t_submit) {
  if (rq.space < DPG_H1 || rq.space > DPG_L2) return fail(DPG_EINVAL, "unknown space %d", rq.space);
  const bool aniso = rq.pdir[0] != 0 || rq.pdir[1] != 0 || rq.pdir[2] != 0;
  int32_t q[3] = {0, 0, 0};
  if (aniso) {
    // non-uniform orders: the per-direction Gram orders, each within the kernels' range
    const int qmax = p_max_ < 10 ? p_max_ : 10;
    for (int d = 0; d < 3; ++d) {
      q[d] = rq.pdir[d] + rq.dp;
      if (rq.pdir[d] < 1 || rq.dp < 0 || q[d] > qmax)
        return fail(DPG_EINVAL, "pdir[%d]=%d dp=%d: Gram order outside [1, %d]", d, rq.pdir[d], rq.dp, qmax);
    }
    if (rq.path == DPG_PATH_REDUCED) return fail(DPG_EINVAL, "non-uniform orders use the quadrature path only");
  } else if (rq.p < 1 || rq.dp < 0 || rq.p + rq.dp > p_max_) {
    return fail(DPG_EINVAL, "p=%d dp=%d: Gram order outside [1, %d]", rq.p, rq.dp, p_max_);
  }
  if (rq.prec != DPG_FP64 && rq.prec != DPG_FP32) return fail(DPG_EINVAL, "unknown precision %d", rq.prec);
  if (rq.path < DPG_PATH_AUTO || rq.path > DPG_PATH_REDUCED) return fail(DPG_EINVAL, "unknown path %d", rq.path);
  if (rq.geom.kind != DPG_GEOM_TRILINEAR && rq.geom.kind != DPG_GEOM_AFFINE && rq.geom.kind != DPG_GEOM_EXTRUDED)
    return fail(DPG_EINVAL, "unknown geometry kind %d", rq.geom.kind);
  if (rq.path == DPG_PATH_REDUCED && rq.geom.kind == DPG_GEOM_TRILINEAR)
    return fail(DPG_EINVAL, "the reduced path needs affine or extruded geometry");
  if (rq.geom.n_elem < 1 || !rq.geom.data) return fail(DPG_EINVAL, "empty request or NULL geometry");
  if (!std::isfinite(rq.w0) || !std::isfinite(rq.w1)) return fail(DPG_EINVAL, "weights must be finite");
  const int pr = aniso ? (q[0] > q[1] ? (q[0] > q[2] ? q[0] : q[2]) : (q[1] > q[2] ? q[1] : q[2])) : rq.p + rq.dp;
  r = Req{};
  r.w.space = rq.space;
  r.w.p = pr;
  for (int d = 0; d < 3; ++d) r.w.q[d] = q[d];
  r.w.prec = rq.prec;
  r.w.path = rq.path;
  r.w.kind = rq.geom.kind;
  r.w.w0 = rq.w0;
  r.w.w1 = rq.w1;
  r.w.n = rq.geom.n_elem;
  if (aniso) {
    int64_t nd = 0;   // component a spans range1d(space, q_d, a, d) functions in direction d
    for (int a = 0; a < ncomp(rq.space); ++a)
      nd += int64_t(range1d(rq.space, q[0], a, 0)) * range1d(rq.space, q[1], a, 1) * range1d(rq.space, q[2], a, 2);
    r.w.packed_len = nd * (nd + 1) / 2;
  } else {
    r.w.packed_len = packed_len(rq.space, pr);
  }
  r.t_submit = t_submit;
  const double bytes = double(r.w.n) * double(r.w.packed_len) * elem_bytes(rq.prec);
  if (bytes > double(out_alloc_.capacity()))
    return fail(DPG_EINVAL, "request output (%.3g bytes) exceeds the memory budget (%lld bytes); split it",
                bytes, (long long)out_alloc_.capacity());
  if (r.w.n > slot_alloc_.capacity())
    return fail(DPG_EINVAL, "request of %lld elements exceeds the %lld element slots", (long long)r.w.n,
                (long long)slot_alloc_.capacity());
  r.out_bytes = out_alloc_.round(int64_t(bytes));
  r.slots = r.w.n;
  return DPG_OK;
}

int Server::enqueue(std::vector<Req>& rs, std::vector<dpg_request>& sub, uint64_t* first) {
  const int64_t k = int64_t(rs.size());
  uint64_t t0;
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return fail(DPG_ENOTINIT, "server is shutting down");
    if (int64_t(queue_.size()) + k > cfg_.max_queue) {
      ++st_rejected_;
      return fail(DPG_EAGAIN, "queue full (%d requests)", cfg_.max_queue);
    }
    int64_t i = 0;
    for (; i < k; ++i) {
      const int64_t s0 = slot_alloc_.alloc(rs[i].slots);
      if (s0 < 0) break;
      rs[i].w.slot0 = s0;
    }
    if (i < k) {   // all or nothing
      for (int64_t j = 0; j < i; ++j) slot_alloc_.release(rs[j].w.slot0, rs[j].slots);
      ++st_rejected_;
      return fail(DPG_EAGAIN, "no %lld free element slots", (long long)rs[i].slots);
    }
    t0 = next_ticket_;
    next_ticket_ += uint64_t(k);
    for (i = 0; i < k; ++i) {
      rs[i].w.ticket = t0 + uint64_t(i);
      rs[i].state = QUEUED;
      reqs_.emplace(t0 + uint64_t(i), rs[i]);   // not in queue_ yet: invisible to the scheduler
    }
  }
  // geometry into the slots, without the lock
  int rc = DPG_OK;
  std::vector<char> staged(size_t(k), 0);
  for (int64_t i = 0; i < k && rc == DPG_OK; ++i) {
    bool st = false;
    rc = ex_->put_geometry(sub[size_t(i)], rs[size_t(i)].w.slot0, &st);
    staged[size_t(i)] = st;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (int64_t i = 0; i < k; ++i) {
      const uint64_t t = t0 + uint64_t(i);
      if (rc != DPG_OK) {
        slot_alloc_.release(rs[size_t(i)].w.slot0, rs[size_t(i)].slots);
        reqs_.erase(t);
        continue;
      }
      reqs_.at(t).w.staged = staged[size_t(i)] != 0;
      queue_.push_back(t);
      ++st_submitted_;
      if (st_first_submit_ < 0) st_first_submit_ = rs[size_t(i)].t_submit;
    }
    if (rc != DPG_OK) {
      ++st_rejected_;
      return rc;
    }
  }
  cv_.notify_one();
  *first = t0;
  return DPG_OK;
}

int Server::submit(const dpg_request& rq, uint64_t* ticket) {
  const double t_submit = now();
  if (!ticket) return fail(DPG_EINVAL, "ticket pointer is NULL");
  *ticket = 0;
  std::vector<Req> rs(1);
  int rc = prepare(rq, rs[0], t_submit);
  if (rc != DPG_OK) {
    std::lock_guard<std::mutex> lk(mu_);
    ++st_rejected_;
    return rc;
  }
  std::vector<dpg_request> sub{rq};
  return enqueue(rs, sub, ticket);
}

int Server::submit_chunked(const dpg_request& rq, int64_t max_chunk_bytes, uint64_t* first, int64_t* n_chunks,
                           int64_t* chunk_elems) {
  const double t_submit = now();
  if (!first || !n_chunks) return fail(DPG_EINVAL, "ticket or chunk-count pointer is NULL");
  *first = 0;
  *n_chunks = 0;
  if (max_chunk_bytes < 0) return fail(DPG_EINVAL, "negative chunk size");
  auto reject = [&](int code) {
    std::lock_guard<std::mutex> lk(mu_);
    ++st_rejected_;
    return code;
  };
  // one element's output against the cap (budget, or the caller's smaller chunk size)
  dpg_request one = rq;
  one.geom.n_elem = rq.geom.n_elem > 0 ? 1 : 0;
  Req probe;
  int rc = prepare(one, probe, t_submit);
  if (rc != DPG_OK) return reject(rc);
  const double per = double(probe.w.packed_len) * elem_bytes(rq.prec);
  const double cap = max_chunk_bytes > 0 ? std::min(double(max_chunk_bytes), double(out_alloc_.capacity()))
                                         : double(out_alloc_.capacity());
  if (per > cap)
    return reject(fail(DPG_EINVAL, "one element's output (%.3g bytes) exceeds the chunk size (%.3g bytes)", per, cap));
  const int64_t ce = std::max<int64_t>(1, std::min<int64_t>(int64_t(cap / per), slot_alloc_.capacity()));
  const int64_t n = rq.geom.n_elem, k = (n + ce - 1) / ce;
  if (k > cfg_.max_queue)
    return reject(fail(DPG_EINVAL, "%lld chunks exceed the queue (%d)", (long long)k, cfg_.max_queue));
  const int64_t stride = rq.geom.kind == DPG_GEOM_TRILINEAR ? 24 : rq.geom.kind == DPG_GEOM_AFFINE ? 12 : 10;
  std::vector<Req> rs(static_cast<size_t>(k));
  std::vector<dpg_request> sub(static_cast<size_t>(k), rq);
  for (int64_t i = 0; i < k; ++i) {
    sub[size_t(i)].geom.data = rq.geom.data + i * ce * stride;
    sub[size_t(i)].geom.n_elem = std::min(ce, n - i * ce);
    rc = prepare(sub[size_t(i)], rs[size_t(i)], t_submit);
    if (rc != DPG_OK) return reject(rc);
  }
  rc = enqueue(rs, sub, first);
  if (rc != DPG_OK) return rc;
  *n_chunks = k;
  if (chunk_elems) *chunk_elems = ce;
  return DPG_OK;
}

void Server::complete_locked(int64_t id, int rc) {
  auto it = launches_.find(id);
  if (it == launches_.end()) return;
  Launch& l = it->second;
  const double t = now();
  for (const Work& w : l.work) {
    auto rit = reqs_.find(w.ticket);
    if (rit == reqs_.end()) continue;
    Req& r = rit->second;
    r.launch = -1;
    r.t_done = t;
    --inflight_reqs_;
    if (rc == 1) {
      r.state = DONE;
      r.status = DPG_OK;
      ++st_completed_;
      st_elements_ += w.n;
      st_bytes_ += double(w.n) * double(w.packed_len) * elem_bytes(w.prec);
      st_last_done_ = t;
      lat_.push_back(r.t_done - r.t_submit);
    } else {
      r.state = FAILED;
      r.status = rc;
      ++st_failed_;
    }
  }
  ex_->retire(l);
  if (l.ids_off >= 0) ids_alloc_.release(l.ids_off, l.items);
  launches_.erase(it);
}

bool Server::sweep_locked() {
  std::vector<std::pair<int64_t, int>> done;
  for (auto& [id, l] : launches_) {
    const int q = ex_->query(l);
    if (q != 0) done.emplace_back(id, q);
  }
  for (auto& [id, q] : done) complete_locked(id, q);
  return !done.empty();
}

void Server::admit_locked() {
  const double t = now();
  while (!queue_.empty() && inflight_reqs_ < cfg_.max_inflight) {
    Req& r = reqs_.at(queue_.front());
    const int64_t off = out_alloc_.alloc(r.out_bytes);
    if (off < 0) break;   // FIFO: later requests wait behind the head
    r.w.out_off = off;
    r.state = RUNNING;
    r.t_admit = t;
    ++inflight_reqs_;
    ++st_admitted_;
    wait_.push_back(r.t_admit - r.t_submit);
    st_peak_bytes_ = std::max(st_peak_bytes_, out_alloc_.used());
    ready_.push_back(queue_.front());
    queue_.pop_front();
  }
}

void Server::launch_locked() {
  if (ready_.empty()) return;
  // group the ready requests by key, in admission order, at most max_merge each
  std::vector<std::vector<uint64_t>> groups;
  for (uint64_t t : ready_) {
    const Work& w = reqs_.at(t).w;
    bool placed = false;
    for (auto& g : groups) {
      if (int(g.size()) < cfg_.max_merge && same_key(reqs_.at(g.front()).w, w)) {
        g.push_back(t);
        placed = true;
        break;
      }
    }
    if (!placed) groups.push_back({t});
  }
  std::vector<uint64_t> deferred;
  for (auto& g : groups) {
    Launch l;
    for (uint64_t t : g) {
      l.work.push_back(reqs_.at(t).w);
      l.items += reqs_.at(t).w.n;
    }
    if (g.size() > 1) {
      l.ids_off = ids_alloc_.alloc(l.items);
      if (l.ids_off < 0) {   // item map space runs out only while launches are on the device
        deferred.insert(deferred.end(), g.begin(), g.end());
        continue;
      }
    }
    // least-loaded stream
    std::vector<int> load(cfg_.n_streams, 0);
    for (auto& [id, x] : launches_) ++load[x.stream];
    l.stream = int(std::min_element(load.begin(), load.end()) - load.begin());
    ++n_launches_started_;
    int rc;
    if (cfg_.test_fail_launch > 0 && n_launches_started_ == cfg_.test_fail_launch)
      rc = fail(DPG_EHIP, "launch %lld failed (test hook)", (long long)n_launches_started_);
    else
      rc = ex_->start(l);
    const int64_t id = next_launch_id_++;
    for (uint64_t t : g) reqs_.at(t).launch = id;
    launches_.emplace(id, std::move(l));
    ++st_launches_;
    st_max_concurrent_ = std::max<int64_t>(st_max_concurrent_, int64_t(launches_.size()));
    if (rc != DPG_OK) complete_locked(id, rc);
  }
  ready_.swap(deferred);
}

void Server::loop() {
  std::unique_lock<std::mutex> lk(mu_);
  while (!stop_) {
    sweep_locked();
    admit_locked();
    launch_locked();
    if (stop_) break;
    if (!launches_.empty() || !ready_.empty())
      // 50 us tick while work is on the device.  system_clock: its timed wait
      // maps to pthread_cond_timedwait (steady_clock's does not everywhere,
      // which thread sanitizers miss); a clock step only delays a tick, and
      // poll() retires finished launches itself.
      cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(50));
    else
      cv_.wait(lk);   // woken by submit, release, completion seen by poll, or stop
  }
}

int Server::poll(uint64_t ticket, dpg_result* res) {
  if (!res) return fail(DPG_EINVAL, "result pointer is NULL");
  bool freed = false;
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return fail(DPG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Req& r = it->second;
  if (r.state == RUNNING && r.launch >= 0) {   // look at the device directly: no scheduler-tick delay
    auto lit = launches_.find(r.launch);
    if (lit != launches_.end()) {
      const int q = ex_->query(lit->second);
      if (q != 0) {
        complete_locked(r.launch, q);
        freed = true;
      }
    }
  }
  if (r.state == QUEUED || r.state == RUNNING) {
    lk.unlock();
    if (freed) cv_.notify_one();
    return DPG_PENDING;
  }
  res->status = r.status;
  res->space = r.w.space;
  res->p = r.w.p;
  res->prec = r.w.prec;
  res->n_elem = r.w.n;
  res->packed_len = r.w.packed_len;
  char* ob = static_cast<char*>(ex_->out_base());
  res->out = (ob && r.state == DONE) ? ob + r.w.out_off : nullptr;
  int32_t* sb = ex_->status_base();
  res->elem_status = (sb && r.state == DONE) ? sb + r.w.slot0 : nullptr;
  res->t_submit = r.t_submit;
  res->t_admit = r.t_admit;
  res->t_done = r.t_done;
  const int status = r.status;
  lk.unlock();
  if (freed) cv_.notify_one();
  return status == DPG_OK ? DPG_OK : fail(status, "request %llu failed (code %d)", (unsigned long long)ticket, status);
}

int Server::read(uint64_t ticket, int what, void* dst, int64_t first, int64_t count, void* stream) {
  Work w;
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail(DPG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state != DONE) return fail(DPG_EINVAL, "request %llu has no result", (unsigned long long)ticket);
    w = it->second.w;
  }
  if (!dst || first < 0 || count < 0 || first + count > w.n)
    return fail(DPG_EINVAL, "read of elements [%lld, %lld) outside [0, %lld)", (long long)first,
                (long long)(first + count), (long long)w.n);
  if (count == 0) return DPG_OK;
  return ex_->copy_out(w, what, first, count, dst, stream);
}

int Server::release(uint64_t ticket) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail(DPG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req& r = it->second;
    if (r.state == RUNNING) return fail(DPG_EAGAIN, "request %llu is on the device", (unsigned long long)ticket);
    if (r.state == QUEUED) {
      auto q = std::find(queue_.begin(), queue_.end(), ticket);
      if (q != queue_.end()) queue_.erase(q);
      ++st_cancelled_;
    } else {
      out_alloc_.release(r.w.out_off, r.out_bytes);
    }
    slot_alloc_.release(r.w.slot0, r.slots);
    reqs_.erase(it);
  }
  cv_.notify_one();
  return DPG_OK;
}

void Server::stats(dpg_serve_stats* s) {
  std::lock_guard<std::mutex> lk(mu_);
  s->submitted = st_submitted_;
  s->rejected = st_rejected_;
  s->admitted = st_admitted_;
  s->completed = st_completed_;
  s->failed = st_failed_;
  s->launches = st_launches_;
  s->cancelled = st_cancelled_;
  s->queued = int64_t(queue_.size());
  s->inflight = inflight_reqs_;
  s->elements = st_elements_;
  s->budget_bytes = out_alloc_.capacity();
  s->admitted_bytes = out_alloc_.used();
  s->peak_admitted_bytes = st_peak_bytes_;
  s->max_concurrent_launches = st_max_concurrent_;
  s->bytes = st_bytes_;
  s->t_first_submit = st_first_submit_ < 0 ? 0.0 : st_first_submit_;
  s->t_last_done = st_last_done_;
  s->lat_p50 = percentile(lat_, 0.50);
  s->lat_p99 = percentile(lat_, 0.99);
  double sum = 0, mx = 0;
  for (double v : lat_) {
    sum += v;
    mx = std::max(mx, v);
  }
  s->lat_mean = lat_.empty() ? 0.0 : sum / double(lat_.size());
  s->lat_max = mx;
  s->wait_p50 = percentile(wait_, 0.50);
  s->wait_p99 = percentile(wait_, 0.99);
}

void Server::reset_stats() {
  std::lock_guard<std::mutex> lk(mu_);
  st_submitted_ = st_rejected_ = st_admitted_ = st_completed_ = st_failed_ = st_cancelled_ = 0;
  st_launches_ = st_elements_ = 0;
  st_peak_bytes_ = out_alloc_.used();
  st_max_concurrent_ = int64_t(launches_.size());
  st_bytes_ = 0;
  st_first_submit_ = -1;
  st_last_done_ = 0;
  lat_.clear();
  wait_.clear();
}

// ---------------------------------------------------------------- timing stub

namespace {

// Stands in for the device in host-side tests of the scheduler: computes
// nothing; each stream is a FIFO that finishes a launch test_launch_s +
// bytes / test_bytes_per_s after the previous one on that stream.
class StubExecutor final : public Executor {
 public:
  explicit StubExecutor(const dpg_serve_cfg& c)
      : rate_(c.test_bytes_per_s > 0 ? c.test_bytes_per_s : 1e12),
        lat_(c.test_launch_s > 0 ? c.test_launch_s : 0.0),
        busy_(c.n_streams, 0.0),
        t0_(std::chrono::steady_clock::now()) {}
  int put_geometry(const dpg_request& req, int64_t, bool*) override {
    return req.geom.data ? DPG_OK : fail(DPG_EINVAL, "NULL geometry");
  }
  int start(Launch& l) override {
    double bytes = 0;
    for (const Work& w : l.work) bytes += double(w.n) * double(w.packed_len) * elem_bytes(w.prec);
    const double t = std::max(clock(), busy_[l.stream]) + lat_ + bytes / rate_;
    busy_[l.stream] = t;
    l.handle = new double(t);
    return DPG_OK;
  }
  int query(Launch& l) override {
    if (!l.handle) return 1;
    return clock() >= *static_cast<double*>(l.handle) ? 1 : 0;
  }
  void retire(Launch& l) override {
    delete static_cast<double*>(l.handle);
    l.handle = nullptr;
  }
  void drain() override {
    const double t = *std::max_element(busy_.begin(), busy_.end());
    while (clock() < t) std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  void* out_base() const override { return nullptr; }
  int32_t* status_base() const override { return nullptr; }
  int copy_out(const Work&, int, int64_t, int64_t, void*, void*) override {
    return fail(DPG_EINVAL, "the test executor produces no results");
  }

 private:
  double clock() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count(); }
  double rate_, lat_;
  std::vector<double> busy_;   // per stream: time its last launch finishes (server lock held)
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace

std::unique_ptr<Executor> make_stub_executor(const dpg_serve_cfg& cfg) {
  return std::make_unique<StubExecutor>(cfg);
}

int check_cfg(const dpg_serve_cfg& c) {
  if (c.mem_budget_bytes < 256) return fail(DPG_EINVAL, "mem_budget_bytes=%lld too small", (long long)c.mem_budget_bytes);
  if (c.max_slots < 1 || c.max_slots > (int64_t(1) << 30))
    return fail(DPG_EINVAL, "max_slots=%lld outside [1, 2^30]", (long long)c.max_slots);
  if (c.max_inflight < 1) return fail(DPG_EINVAL, "max_inflight must be positive");
  if (c.max_queue < 1) return fail(DPG_EINVAL, "max_queue must be positive");
  if (c.n_streams < 1 || c.n_streams > 8) return fail(DPG_EINVAL, "n_streams=%d outside [1, 8]", c.n_streams);
  if (c.max_merge < 1 || c.max_merge > kMaxMerge)
    return fail(DPG_EINVAL, "max_merge=%d outside [1, %d]", c.max_merge, kMaxMerge);
  if (c.test_executor != 0 && c.test_executor != 1) return fail(DPG_EINVAL, "unknown test_executor %d", c.test_executor);
  return DPG_OK;
}

}  // namespace dpg::serve
