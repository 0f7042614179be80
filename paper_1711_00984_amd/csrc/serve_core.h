// serve_core.h -- host side of the serving loop: admission, continuous
// batching, request bookkeeping and latency statistics.  Pure C++ (no HIP):
// the device work goes through the Executor interface, implemented with HIP
// streams and events in serve.cpp and by a timing stub for host-side tests.
//
// Life of a request (ticket):
//   submit   -> element slots reserved, geometry copied into them, QUEUED
//   admit    -> output bytes reserved in the output arena (FIFO; stops at the
//               first request that does not fit), RUNNING
//   launch   -> requests admitted in the same scheduler pass with the same
//               (space, order, precision, path, geometry kind, weights) share
//               one launch; launches go out on several streams and overlap
//               with the work already on the device
//   complete -> DONE (or FAILED), result pollable
//   release  -> output bytes and slots returned; waiting requests get admitted
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dpg.h"

namespace dpg::serve {

constexpr int kMaxMerge = 32;   // requests per launch (item-map kernel argument size)

// First-fit allocator over [0, capacity) with coalescing of freed ranges.
// Sizes and offsets are multiples of `align`.  Not thread-safe (the server
// holds its mutex).
class RangeAlloc {
 public:
  RangeAlloc() = default;
  RangeAlloc(int64_t capacity, int64_t align);
  int64_t alloc(int64_t n);            // offset, or -1 if no free range fits
  void release(int64_t off, int64_t n);
  int64_t capacity() const { return cap_; }
  int64_t used() const { return used_; }
  int64_t round(int64_t n) const { return (n + align_ - 1) / align_ * align_; }

 private:
  int64_t cap_ = 0, align_ = 1, used_ = 0;
  std::map<int64_t, int64_t> free_;    // offset -> length
};

// One admitted request as the executor sees it.
struct Work {
  uint64_t ticket = 0;
  int space = 0, p = 0, prec = 0, path = 0, kind = 0;
  int q[3] = {0, 0, 0};    // non-uniform Gram orders per direction (zeros: the uniform order p)
  double w0 = 1, w1 = 1;
  int64_t n = 0;           // elements
  int64_t slot0 = 0;       // first element slot (geometry, status)
  int64_t out_off = 0;     // byte offset of the output in the output arena
  int64_t packed_len = 0;
  bool staged = false;     // geometry waits in host staging; the launch uploads it
};

// A launch: requests with one key, ids_off = start of its item->slot map.
struct Launch {
  std::vector<Work> work;
  int64_t items = 0;
  int64_t ids_off = -1;
  int stream = 0;
  void* handle = nullptr;  // executor's completion token
};

class Executor {
 public:
  virtual ~Executor() = default;
  // Take a copy of a request's geometry for its slots (called at submit,
  // without the server lock).  Device geometry is copied into the slots before
  // this returns; host geometry may instead be staged in host memory
  // (*staged = true), and start() then uploads it ahead of the kernels.
  virtual int put_geometry(const dpg_request& req, int64_t slot0, bool* staged) = 0;
  // Enqueue the launch; on success l.handle is set.
  virtual int start(Launch& l) = 0;
  // 1 finished, 0 still running, < 0 error code (the launch failed).
  virtual int query(Launch& l) = 0;
  // Free per-launch resources after query() returned non-zero.
  virtual void retire(Launch& l) = 0;
  // Block until every started launch has finished.
  virtual void drain() = 0;
  virtual void* out_base() const = 0;
  virtual int32_t* status_base() const = 0;
  // Copy elements [first, first + count) of a result (what 0: output
  // entries, 1: status words) to dst, asynchronously on stream.
  virtual int copy_out(const Work& w, int what, int64_t first, int64_t count, void* dst, void* stream) = 0;
};

class Server {
 public:
  Server(const dpg_serve_cfg& cfg, int p_max, std::unique_ptr<Executor> ex);
  ~Server();
  int submit(const dpg_request& req, uint64_t* ticket);
  // A request cut into element chunks whose output fits max_chunk_bytes (0: the budget),
  // queued as consecutive tickets, all or none.
  int submit_chunked(const dpg_request& req, int64_t max_chunk_bytes, uint64_t* first, int64_t* n_chunks,
                     int64_t* chunk_elems);
  int poll(uint64_t ticket, dpg_result* res);
  int release(uint64_t ticket);
  int read(uint64_t ticket, int what, void* dst, int64_t first, int64_t count, void* stream);
  void stats(dpg_serve_stats* st);
  void reset_stats();

 private:
  enum State { QUEUED, RUNNING, DONE, FAILED };
  struct Req {
    Work w;
    State state = QUEUED;
    int status = DPG_OK;
    int64_t out_bytes = 0;   // rounded reservation in the output arena
    int64_t slots = 0;       // rounded reservation in the slot arena
    int64_t launch = -1;     // key in launches_ while on the device
    double t_submit = 0, t_admit = 0, t_done = 0;
  };

  // validate a request and size its reservations (no lock)
  int prepare(const dpg_request& rq, Req& r, double t_submit);
  // reserve slots and consecutive tickets for rs (all or none), copy each geometry
  // (sub[i]) into its slots, then queue them in order; *first = the first ticket
  int enqueue(std::vector<Req>& rs, std::vector<dpg_request>& sub, uint64_t* first);
  void loop();
  void complete_locked(int64_t id, int rc);
  bool sweep_locked();
  void admit_locked();
  void launch_locked();
  double now() const;

  dpg_serve_cfg cfg_;
  int p_max_;
  std::unique_ptr<Executor> ex_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  RangeAlloc out_alloc_, slot_alloc_, ids_alloc_;
  std::unordered_map<uint64_t, Req> reqs_;
  std::deque<uint64_t> queue_;         // QUEUED, in submit order
  std::vector<uint64_t> ready_;        // admitted, not yet launched
  std::map<int64_t, Launch> launches_; // on the device, by launch id
  int64_t next_launch_id_ = 0;
  uint64_t next_ticket_ = 1;
  int64_t n_launches_started_ = 0;
  int inflight_reqs_ = 0;
  // statistics
  int64_t st_submitted_ = 0, st_rejected_ = 0, st_admitted_ = 0, st_completed_ = 0, st_failed_ = 0;
  int64_t st_cancelled_ = 0;
  int64_t st_launches_ = 0, st_elements_ = 0, st_peak_bytes_ = 0, st_max_concurrent_ = 0;
  double st_bytes_ = 0, st_first_submit_ = -1, st_last_done_ = 0;
  std::vector<double> lat_, wait_;
  std::chrono::steady_clock::time_point t0_;
  std::thread thr_;
};

// Validate a configuration (0 or a DPG_E* code with the message set).
int check_cfg(const dpg_serve_cfg& cfg);
// The timing stub behind cfg.test_executor = 1.
std::unique_ptr<Executor> make_stub_executor(const dpg_serve_cfg& cfg);

}  // namespace dpg::serve
