// Serving: continuous batching of independent hybrid solves on one GPU.
//
// The server owns one device arena of the HBM budget, allocated once, so no
// device allocation or free happens while requests run.  max_slots worker
// threads each own a HIP stream (default priority).  A worker takes the first
// queued request, in arrival order, whose footprint fits in the arena (a
// request that does not fit yet is passed over, not dropped), creates its
// solver inside a bump-allocated block of the arena on the worker's stream,
// runs all of its time steps, copies out phi_R, the balance and the latency
// record, and returns the block.  Requests therefore enter as soon as a slot
// and memory are free, and the kernels of concurrently resident requests
// overlap on the device through their streams.  Each solve's sums are
// order-independent fixed point, so a request's result does not depend on
// what else runs beside it.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/slh.h"

namespace slh {
void set_last_error(const std::string& msg);
}

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over the arena, with coalescing of free neighbours.
class Arena {
 public:
  bool init(size_t bytes) {
    if (hipMalloc(&base_, bytes) != hipSuccess) { base_ = nullptr; return false; }
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  void release() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
    free_.clear();
  }
  // returns offset or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void free(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return (char*)base_; }
  size_t size() const { return size_; }

 private:
  static constexpr size_t kAlign = 4096;
  void* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_, used_;
};

enum ReqState { Q_QUEUED = 0, Q_RUNNING, Q_DONE };

struct Request {
  uint64_t ticket = 0;
  slh_problem prob;
  std::vector<double> ss, sa, q;
  std::vector<int32_t> ns;  // per-cell scatter limits, if given
  std::vector<double> inflow;  // boundary inflow, if given
  int n_steps = 0;
  size_t footprint = 0;
  ReqState state = Q_QUEUED;
  slh_status status = SLH_OK;
  std::string error;
  std::vector<double> flux;
  slh_balance bal;
  slh_latency lat;
  // arena block
  size_t block_off = SIZE_MAX, block_len = 0, bump = 0;
  char* block_base = nullptr;
};

// Bump allocation inside a request's arena block.
void* block_alloc(size_t bytes, void* ctx) {
  Request* r = (Request*)ctx;
  const size_t a = 256;
  size_t off = (r->bump + a - 1) / a * a;
  if (off + bytes > r->block_len) return nullptr;
  r->bump = off + bytes;
  return r->block_base + off;
}
void block_free(void*, void*) {}

}  // namespace

struct slh_server {
  slh_server_cfg cfg;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> reqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  uint64_t next_ticket = 1;
  bool stop = false;
  int device = 0;
  // requests admitted ahead of the one at the head of the queue since it
  // became the head
  int head_bypass = 0;
};

// How many later requests may be admitted ahead of the head of the queue
// while it does not fit; after that the arena is held for it.
constexpr int kMaxHeadBypass = 4;


// Finds the first queued request whose block fits, in arrival order, except
// that once kMaxHeadBypass later requests have been admitted ahead of the
// head of the queue only the head is (so a large request cannot starve
// behind a stream of small ones); called with mu held.
static Request* take_admissible(slh_server* srv) {
  for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
    Request* r = *it;
    const bool head = it == srv->queue.begin();
    if (!head && srv->head_bypass >= kMaxHeadBypass) break;
    const size_t off = srv->arena.alloc(r->footprint);
    if (off != SIZE_MAX) {
      r->block_off = off;
      r->block_len = r->footprint;
      r->block_base = srv->arena.base() + off;
      r->bump = 0;
      srv->queue.erase(it);
      srv->head_bypass = head ? 0 : srv->head_bypass + 1;
      return r;
    }
  }
  return nullptr;
}

static void run_request(Request* r, hipStream_t stream) {
  slh_solver* s = nullptr;
  r->status = slh_create(&r->prob, stream, block_alloc, block_free, r, &s);
  if (r->status != SLH_OK) {
    r->error = slh_last_error();
    return;
  }
  slh_status st = slh_advance(s, r->n_steps);
  if (st == SLH_OK) st = slh_synchronize(s);  // the steps' outcome
  if (st != SLH_OK && st != SLH_E_NOT_CONVERGED) {
    r->status = st;
    r->error = slh_last_error();
    slh_destroy(s);
    return;
  }
  r->status = st;
  r->flux.resize((size_t)r->prob.nx * r->prob.ny);
  slh_status g = slh_get_flux(s, SLH_FLUX_REMAP, r->flux.data());
  if (g == SLH_OK) g = slh_get_balance(s, 2, &r->bal);
  slh_stats stats;
  if (g == SLH_OK) g = slh_get_stats(s, &stats);
  if (g != SLH_OK) {
    r->status = g;
    r->error = slh_last_error();
  } else {
    r->lat.segments = stats.seg_mc_total + stats.seg_remap_total;
  }
  slh_destroy(s);
}

static void worker_main(slh_server* srv, int w) {
  (void)hipSetDevice(srv->device);
  hipStream_t stream = srv->streams[w];
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      for (;;) {
        if (!srv->queue.empty()) {
          r = take_admissible(srv);
          if (r) break;
        }
        if (srv->stop && srv->queue.empty()) return;
        srv->cv.wait(lk);
      }
      r->state = Q_RUNNING;
      r->lat.admit_s = now_s();
    }
    run_request(r, stream);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->arena.free(r->block_off);
      r->lat.done_s = now_s();
      r->lat.queue_ms = 1e3 * (r->lat.admit_s - r->lat.submit_s);
      r->lat.run_ms = 1e3 * (r->lat.done_s - r->lat.admit_s);
      r->lat.latency_ms = 1e3 * (r->lat.done_s - r->lat.submit_s);
      r->state = Q_DONE;
    }
    srv->cv.notify_all();
  }
}

extern "C" slh_status slh_server_create(const slh_server_cfg* cfg, slh_server** out) {
  if (!out) return SLH_E_INVALID_ARG;
  *out = nullptr;
  slh_server* srv = new (std::nothrow) slh_server();
  if (!srv) return SLH_E_OUT_OF_MEMORY;
  srv->cfg.hbm_budget_bytes = cfg && cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes
                                                           : ((size_t)64 << 30);
  srv->cfg.max_slots = cfg && cfg->max_slots > 0 ? cfg->max_slots : 8;
  srv->cfg.n_streams = srv->cfg.max_slots;  // one stream per slot
  if (srv->cfg.max_slots > 64) {
    delete srv;
    return SLH_E_INVALID_ARG;
  }
  (void)hipGetDevice(&srv->device);
  if (!srv->arena.init(srv->cfg.hbm_budget_bytes)) {
    delete srv;
    return SLH_E_OUT_OF_MEMORY;
  }
  for (int w = 0; w < srv->cfg.max_slots; ++w) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto t : srv->streams) (void)hipStreamDestroy(t);
      srv->arena.release();
      delete srv;
      return SLH_E_DEVICE;
    }
    srv->streams.push_back(s);
  }
  for (int w = 0; w < srv->cfg.max_slots; ++w)
    srv->workers.emplace_back(worker_main, srv, w);
  *out = srv;
  return SLH_OK;
}

extern "C" slh_status slh_server_submit(slh_server* srv, const slh_problem* p, int32_t n_steps,
                                        uint64_t* ticket) {
  if (!srv || !p || !ticket || n_steps < 1) return SLH_E_INVALID_ARG;
  const size_t fp = slh_footprint_bytes(p);  // validates the parameters
  if (fp == 0) return SLH_E_INVALID_ARG;
  if (!p->sigma_s || !p->sigma_a || !p->q) return SLH_E_INVALID_ARG;
  if (fp > srv->arena.size()) return SLH_E_REJECTED;
  Request* r = new (std::nothrow) Request();
  if (!r) return SLH_E_OUT_OF_MEMORY;
  const size_t n = (size_t)p->nx * p->ny;
  r->prob = *p;
  r->ss.assign(p->sigma_s, p->sigma_s + n);
  r->sa.assign(p->sigma_a, p->sigma_a + n);
  r->q.assign(p->q, p->q + n);
  r->prob.sigma_s = r->ss.data();
  r->prob.sigma_a = r->sa.data();
  r->prob.q = r->q.data();
  if (p->n_s_cell) {
    r->ns.assign(p->n_s_cell, p->n_s_cell + n);
    r->prob.n_s_cell = r->ns.data();
  }
  if (p->inflow) {
    r->inflow.assign(p->inflow, p->inflow + 2 * ((size_t)p->nx + p->ny));
    r->prob.inflow = r->inflow.data();
  }
  r->n_steps = n_steps;
  r->footprint = fp;
  memset(&r->bal, 0, sizeof(r->bal));
  memset(&r->lat, 0, sizeof(r->lat));
  r->lat.submit_s = now_s();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    srv->reqs[r->ticket] = r;
    srv->queue.push_back(r);
    *ticket = r->ticket;
  }
  srv->cv.notify_all();
  return SLH_OK;
}

extern "C" slh_status slh_server_poll(slh_server* srv, uint64_t ticket, int32_t* done) {
  if (!srv || !done) return SLH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return SLH_E_INVALID_ARG;
  *done = it->second->state == Q_DONE ? 1 : 0;
  return SLH_OK;
}

extern "C" slh_status slh_server_result(slh_server* srv, uint64_t ticket, double* flux_out,
                                        slh_balance* balance, slh_latency* latency) {
  if (!srv) return SLH_E_INVALID_ARG;
  Request* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SLH_E_INVALID_ARG;
    r = it->second;
    srv->cv.wait(lk, [&] { return r->state == Q_DONE; });
    srv->reqs.erase(it);
  }
  const slh_status st = r->status;
  if (st != SLH_OK) slh::set_last_error(r->error);
  if (flux_out && !r->flux.empty()) memcpy(flux_out, r->flux.data(), 8 * r->flux.size());
  if (balance) *balance = r->bal;
  if (latency) *latency = r->lat;
  delete r;
  return st;
}

extern "C" void slh_server_destroy(slh_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  for (auto& t : srv->workers) t.join();
  for (auto& kv : srv->reqs) delete kv.second;
  for (auto s : srv->streams) (void)hipStreamDestroy(s);
  srv->arena.release();
  delete srv;
}
