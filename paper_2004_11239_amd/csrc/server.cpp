// Request server with continuous batching for the collision operator.
//
// A request asks for Q(f) of one homogeneous cell (eq. realQ) or to advance
// it by n_steps Heun steps (2 evaluations each) under given (N, L, R, gamma,
// s, N_rho, M, precision).  Requests arrive from any host thread
// (bzq_server_submit; refused with BZQ_EBUSY when the bounded queue is full)
// and are served by one worker thread that owns every HIP call:
//   * plans are cached by their parameters and kept resident; a plan's
//     workspaces are pooled, so concurrent requests on one plan each get
//     their own scratch; plans that differ only in gamma share one set of
//     tables (gamma enters only through c_p), counted once in the budget;
//   * admission is by device-memory footprint: a request starts only when
//     its plan (if not cached), a workspace (if none is free) and its state
//     fit in the budget; idle cached plans are evicted least recently used
//     first; a request waits for memory only while other requests run (whose
//     completion frees some), otherwise it fails with ENOMEM;
//   * up to `slots` requests run at once, each on its own stream, so their
//     kernels overlap on the device; a finishing request frees its slot and
//     memory and the next queued requests are admitted at once (FIFO order);
//   * times (arrival, start, completion) are taken on the host's monotonic
//     clock; completion is detected by polling a HIP event per slot.
// Each request runs the same kernels in the same order as bzq_step on a
// fresh workspace, so its result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "plan.hpp"

using namespace bzq;

namespace {

using Clock = std::chrono::steady_clock;

struct PlanEntry {
  std::string key;
  std::string tkey;                 // the plan's gamma-independent tables
  bzq_plan plan = nullptr;
  bool tuned = false;               // schedule timed (BZQ_SERVER_TUNE) or inherited
  size_t plan_bytes = 0;            // excluding the shared tables
  size_t ws_bytes = 0;              // bytes of one extra workspace
  int in_use = 0;
  bool own_ws_busy = false;         // the plan's built-in workspace
  std::vector<Workspace*> free_ws;  // extra workspaces not in use
  std::vector<Workspace*> all_ws;
  double last_used = 0;
};

struct Request {
  unsigned long long id = 0;
  bzq_request desc{};
  std::vector<double> host_f;       // input, then the result
  double t_arrival = 0, t_start = 0, t_done = 0;
  int state = 0;                    // 0 queued, 1 running, 2 done, 3 failed
  bzq_status err = BZQ_OK;
  std::string msg;
  // resources while running
  PlanEntry* pe = nullptr;
  Workspace* ws = nullptr;          // nullptr: the plan's own workspace
  double* d_f = nullptr;
  double* h_pin = nullptr;
  size_t charged = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Request* req = nullptr;
};

}  // namespace

struct bzq_server_s {
  int device = 0;
  size_t budget = 0;
  int max_queued = 0;               // 0: unbounded
  int flags = 0;
  size_t used = 0, peak = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> incoming;                   // guarded by mu
  std::unordered_map<unsigned long long, std::unique_ptr<Request>> reqs;   // guarded by mu
  std::deque<Request*> pending;                    // worker only
  std::map<std::string, std::unique_ptr<PlanEntry>> plans;   // worker only
  std::map<std::string, std::pair<size_t, int>> tables;       // tkey -> (bytes, plans holding them)
  std::map<int, std::vector<std::pair<double*, double*>>> buf_pool;   // N -> (device f, pinned host)
  std::thread worker;
  std::atomic<bool> stop{false};
  unsigned long long next_id = 1;
  Clock::time_point t0 = Clock::now();
  // stats (guarded by mu)
  unsigned long long submitted = 0, completed = 0, failed = 0, evictions = 0, rejected = 0;
  int running = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

std::string plan_key(const bzq_request& d) {
  std::ostringstream k;
  k.precision(17);
  k << d.N << "|" << d.L << "|" << d.R << "|" << d.gamma << "|" << d.s << "|" << d.N_rho << "|" << d.M << "|"
    << d.precision;
  return k.str();
}

// plans that differ only in gamma share their tables (bzq_plan_derive_gamma)
std::string table_key(const bzq_request& d) {
  std::ostringstream k;
  k.precision(17);
  k << d.N << "|" << d.L << "|" << d.R << "|" << d.s << "|" << d.N_rho << "|" << d.M << "|" << d.precision;
  return k.str();
}



void release_plan(bzq_server_s* s, PlanEntry* pe) {
  for (Workspace* w : pe->all_ws) delete w;
  s->used -= pe->plan_bytes + pe->ws_bytes * pe->all_ws.size();
  bzq_plan_destroy(pe->plan);
  auto t = s->tables.find(pe->tkey);
  if (t != s->tables.end() && --t->second.second == 0) {
    s->used -= t->second.first;
    s->tables.erase(t);
  }
}

// make room for `need` bytes by evicting idle plans, least recently used first
bool make_room(bzq_server_s* s, size_t need, const PlanEntry* keep) {
  while (s->used + need > s->budget) {
    PlanEntry* victim = nullptr;
    for (auto& kv : s->plans) {
      PlanEntry* pe = kv.second.get();
      if (pe == keep || pe->in_use > 0) continue;
      if (!victim || pe->last_used < victim->last_used) victim = pe;
    }
    if (!victim) return false;
    release_plan(s, victim);
    s->plans.erase(victim->key);
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->evictions;
  }
  return true;
}

void finish(bzq_server_s* s, Request* r, int state, bzq_status err, const std::string& msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->state = state;
  r->err = err;
  r->msg = msg;
  r->t_done = s->now();
  if (state == 2) ++s->completed; else ++s->failed;
  s->cv_done.notify_all();
}

// Try to start r on slot sl.  Returns false when the memory budget does not
// allow it yet (r stays queued); failures are reported on r.
bool try_start(bzq_server_s* s, Request* r, Slot& sl) {
  const bzq_request& d = r->desc;
  const std::string key = plan_key(d);
  PlanEntry* pe = nullptr;
  auto it = s->plans.find(key);
  if (it == s->plans.end()) {
    // a new plan: its footprint is known from the geometry before creating
    // it; a cached plan differing only in gamma lends its tables
    const std::string tkey = table_key(d);
    PlanEntry* base = nullptr;
    for (auto& kv : s->plans)
      if (kv.second->tkey == tkey) {
        base = kv.second.get();
        break;
      }
    const size_t full = plan_footprint(d.N, d.N_rho, d.M, d.precision) + state_bytes(d.N);
    const size_t est = base ? full - plan_shared_bytes_estimate(d.N, d.N_rho, d.M, d.precision) : full;
    if (full > s->budget) {
      finish(s, r, 3, BZQ_ENOMEM, "request does not fit the device-memory budget");
      return true;
    }
    if (s->used + est > s->budget && !make_room(s, est, base)) {
      // no room beside the plan that would lend its tables: build a plan of
      // its own instead, with that one evictable too
      if (!base || !make_room(s, full, nullptr)) {
        if (s->running == 0) {
          finish(s, r, 3, BZQ_ENOMEM, "request does not fit the device-memory budget beside the cached plans");
          return true;
        }
        return false;   // a completion will free memory
      }
      base = nullptr;
    }
    bzq_plan p = nullptr;
    bzq_status st;
    if (base) {
      st = derive_plan(*base->plan, d.gamma, &p, sl.stream);
    } else {
      const double bc = power_kernel_constant(d.s);
      st = create_plan(&p, d.N, d.L, d.R, d.gamma, bc, d.s, 0.0, 64, d.N_rho, d.M, d.precision, sl.stream);
    }
    if (st != BZQ_OK) {
      if (st == BZQ_ENOMEM && s->running > 0) return false;   // retry once memory is freed
      finish(s, r, 3, st, bzq_last_error());
      return true;
    }
    const size_t shared = bzq_plan_shared_bytes(p);
    const size_t pb = bzq_plan_device_bytes(p) - shared;
    auto e = std::make_unique<PlanEntry>();
    e->key = key;
    e->tkey = tkey;
    e->plan = p;
    e->plan_bytes = pb;
    e->ws_bytes = p->ws.arena.bytes;
    e->tuned = base != nullptr;       // a derived plan inherits its base's schedule
    s->used += pb;
    auto& t = s->tables[tkey];
    if (t.second++ == 0) {
      t.first = shared;
      s->used += shared;
    }
    pe = e.get();
    s->plans[key] = std::move(e);
  } else {
    pe = it->second.get();
  }
  // workspace: the plan's own if free, else a pooled one, else a new one
  Workspace* ws = nullptr;
  bool own = false;
  size_t need = 0;
  if (!pe->own_ws_busy) {
    own = true;
  } else if (!pe->free_ws.empty()) {
    ws = pe->free_ws.back();
  } else {
    need += pe->ws_bytes;
  }
  auto bit = s->buf_pool.find(d.N);
  const bool have_buf = bit != s->buf_pool.end() && !bit->second.empty();
  if (!have_buf) need += state_bytes(d.N);
  if (need && s->used + need > s->budget && !make_room(s, need, pe)) {
    if (s->running == 0 && pe->in_use == 0) {
      finish(s, r, 3, BZQ_ENOMEM, "request does not fit the device-memory budget");
      return true;
    }
    return false;
  }
  // an allocation that fails while nothing runs would fail again: the
  // request fails instead of waiting for a completion that never comes
  auto alloc_failed = [&](const char* what) {
    if (s->running == 0 && pe->in_use == 0) {
      finish(s, r, 3, BZQ_ENOMEM, std::string("allocation of the request's ") + what + " failed");
      return true;
    }
    return false;
  };
  if (!own && !ws) {
    ws = new Workspace();
    if (workspace_init(*ws, *pe->plan, 1) != BZQ_OK) {
      delete ws;
      return alloc_failed("workspace");
    }
    pe->all_ws.push_back(ws);
    s->used += pe->ws_bytes;
  } else if (ws) {
    pe->free_ws.pop_back();
  }
  double* d_f = nullptr;
  double* h_pin = nullptr;
  if (have_buf) {
    d_f = bit->second.back().first;
    h_pin = bit->second.back().second;
    bit->second.pop_back();
  } else {
    if (hipMalloc(&d_f, state_bytes(d.N)) != hipSuccess) {
      (void)hipGetLastError();
      if (ws) pe->free_ws.push_back(ws);
      return alloc_failed("state");
    }
    if (hipHostMalloc(&h_pin, state_bytes(d.N), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(d_f);
      if (ws) pe->free_ws.push_back(ws);
      return alloc_failed("pinned host buffer");
    }
    s->used += state_bytes(d.N);
  }
  s->peak = std::max(s->peak, s->used);
  if (own) pe->own_ws_busy = true;
  ++pe->in_use;
  pe->last_used = s->now();
  r->pe = pe;
  r->ws = own ? nullptr : ws;
  r->d_f = d_f;
  r->h_pin = h_pin;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->state = 1;
    r->t_start = s->now();
    ++s->running;
  }
  std::memcpy(h_pin, r->host_f.data(), state_bytes(d.N));
  Workspace& w = own ? pe->plan->ws : *ws;
  hipError_t e1 = hipMemcpyAsync(d_f, h_pin, state_bytes(d.N), hipMemcpyHostToDevice, sl.stream);
  bzq_status st = e1 == hipSuccess ? BZQ_OK : BZQ_EDEVICE;
  if (st == BZQ_OK && (s->flags & BZQ_SERVER_TUNE) && !pe->tuned) {
    // the first request of a new plan: time its schedule on this input
    // (synchronous, on the plan's own workspace, before the request runs)
    pe->tuned = true;
    if (own) st = bzq_plan_autotune(pe->plan, d_f, 1, sl.stream);
  }
  // the result: the new state (step) or Q(f) in the workspace's stage buffer
  double* result = d_f;
  if (st == BZQ_OK) {
    if (d.kind == BZQ_REQ_COLLISION) {
      result = w.q1;
      st = enqueue_collision(*pe->plan, w, single(d_f), single(result), 1, sl.stream);
    } else {
      st = enqueue_step(*pe->plan, w, single(d_f), 1, d.dt, d.n_steps, sl.stream);
    }
  }
  hipError_t e2 = st == BZQ_OK ? hipMemcpyAsync(h_pin, result, state_bytes(d.N), hipMemcpyDeviceToHost, sl.stream)
                               : hipErrorUnknown;
  if (e2 != hipSuccess && st == BZQ_OK) st = BZQ_EDEVICE;
  // the event is recorded after whatever was enqueued, also on failure, so
  // that the request's buffers return to the pools only once its kernels end
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipEventRecord(sl.done, nullptr);
    if (st == BZQ_OK) st = BZQ_EDEVICE;
  }
  r->err = st;
  sl.req = r;
  return true;
}

void complete(bzq_server_s* s, Slot& sl) {
  Request* r = sl.req;
  sl.req = nullptr;
  PlanEntry* pe = r->pe;
  const int N = r->desc.N;
  if (r->err == BZQ_OK) std::memcpy(r->host_f.data(), r->h_pin, state_bytes(N));
  if (r->ws) pe->free_ws.push_back(r->ws); else pe->own_ws_busy = false;
  --pe->in_use;
  pe->last_used = s->now();
  s->buf_pool[N].push_back({r->d_f, r->h_pin});
  {
    std::lock_guard<std::mutex> lk(s->mu);
    --s->running;
  }
  if (r->err == BZQ_OK) finish(s, r, 2, BZQ_OK, "");
  else finish(s, r, 3, r->err, "device error while running the request");
}

void worker_main(bzq_server_s* s) {
  (void)hipSetDevice(s->device);
  bool blocked = false;   // the queue's head waits for memory (only while requests run)
  while (!s->stop.load()) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
    }
    bool progressed = false;
    for (Slot& sl : s->slots) {
      if (sl.req && hipEventQuery(sl.done) == hipSuccess) {
        complete(s, sl);
        progressed = true;
        blocked = false;                      // memory was freed
      }
    }
    if (s->running == 0) blocked = false;   // nothing left to wait for
    for (Slot& sl : s->slots) {
      if (blocked || sl.req || s->pending.empty()) continue;
      Request* r = s->pending.front();
      if (!try_start(s, r, sl)) {             // keep FIFO order: wait for memory
        blocked = true;
        break;
      }
      s->pending.pop_front();
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(200), [&] { return s->stop.load() || !s->incoming.empty(); });
    }
  }
}

}  // namespace

extern "C" {

bzq_status bzq_server_create(bzq_server* out, size_t budget_bytes, int slots, int max_queued, int flags) {
  if (!out) return fail(BZQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (slots < 1 || slots > 16) return fail(BZQ_EINVAL, "slots must lie in [1, 16]");
  if (budget_bytes < (64ull << 20)) return fail(BZQ_EINVAL, "budget below 64 MiB");
  if (max_queued < 0) return fail(BZQ_EINVAL, "max_queued must be >= 0");
  if (flags & ~BZQ_SERVER_TUNE) return fail(BZQ_EINVAL, "unknown server flag");
  auto* s = new bzq_server_s();
  s->budget = budget_bytes;
  s->max_queued = max_queued;
  s->flags = flags;
  BZQ_HIP_TRY(hipGetDevice(&s->device));
  s->slots.resize(slots);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      delete s;
      return fail(BZQ_EDEVICE, "stream or event creation failed");
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return BZQ_OK;
}

bzq_status bzq_server_submit(bzq_server s, const bzq_request* req, const double* f_host, unsigned long long* id) {
  if (!s || !req || !f_host || !id) return fail(BZQ_EINVAL, "NULL argument");
  const int N = req->N;
  if (N < 8 || (N & 1)) return fail(BZQ_EINVAL, "N must be even and >= 8");
  if (!supported_N(N)) return fail(BZQ_EUNSUPPORTED, "no FFT schedule for this N (supported: 8 16 24 32 48 64 128)");
  if (req->kind != BZQ_REQ_STEP && req->kind != BZQ_REQ_COLLISION) return fail(BZQ_EINVAL, "unknown request kind");
  if (req->kind == BZQ_REQ_STEP && (req->n_steps < 0 || !std::isfinite(req->dt)))
    return fail(BZQ_EINVAL, "bad dt or n_steps");
  if (s->max_queued > 0) {
    std::lock_guard<std::mutex> lk(s->mu);
    const unsigned long long queued = s->submitted - s->completed - s->failed - (unsigned long long)s->running;
    if (queued >= (unsigned long long)s->max_queued) {
      ++s->rejected;
      return fail(BZQ_EBUSY, "request queue full");
    }
  }
  auto r = std::make_unique<Request>();
  r->desc = *req;
  r->host_f.assign(f_host, f_host + (size_t)N * N * N * 2);
  Request* raw = r.get();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->t_arrival = s->now();
    *id = r->id;
    s->reqs[r->id] = std::move(r);
    s->incoming.push_back(raw);
    ++s->submitted;
  }
  s->cv_work.notify_one();
  return BZQ_OK;
}

int bzq_server_poll(bzq_server s, unsigned long long id, double* f_out, double* times) {
  if (!s) return -1;
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return -1;
    if (it->second->state < 2) return 0;
    r = std::move(it->second);
    s->reqs.erase(it);
  }
  if (times) {
    times[0] = r->t_arrival;
    times[1] = r->t_start;
    times[2] = r->t_done;
  }
  if (r->state == 3) {
    fail(r->err, r->msg);
    return -2;
  }
  if (f_out) std::memcpy(f_out, r->host_f.data(), r->host_f.size() * sizeof(double));
  return 1;
}

bzq_status bzq_server_wait(bzq_server s, unsigned long long id, double timeout_s) {
  if (!s) return fail(BZQ_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->reqs.find(id);
    return it == s->reqs.end() || it->second->state >= 2;
  };
  if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
    return fail(BZQ_EDEVICE, "timed out waiting for the request");
  return BZQ_OK;
}

bzq_status bzq_server_stats(bzq_server s, double* out) {
  if (!s || !out) return fail(BZQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out[0] = (double)s->submitted;
  out[1] = (double)s->completed;
  out[2] = (double)s->failed;
  out[3] = (double)(s->submitted - s->completed - s->failed - s->running);
  out[4] = (double)s->running;
  out[5] = (double)s->used;
  out[6] = (double)s->peak;
  out[7] = (double)s->evictions;
  out[8] = (double)s->rejected;
  return BZQ_OK;
}

bzq_status bzq_server_destroy(bzq_server s) {
  if (!s) return BZQ_OK;
  s->stop.store(true);
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipDeviceSynchronize();
  for (auto& kv : s->plans) {
    for (Workspace* w : kv.second->all_ws) delete w;
    bzq_plan_destroy(kv.second->plan);
  }
  for (auto& kv : s->buf_pool)
    for (auto& b : kv.second) {
      (void)hipFree(b.first);
      (void)hipHostFree(b.second);
    }
  for (Slot& sl : s->slots) {
    if (sl.req && sl.req->d_f) {
      (void)hipFree(sl.req->d_f);
      (void)hipHostFree(sl.req->h_pin);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return BZQ_OK;
}

}  // extern "C"
