// Serving: many registrations resident on one GPU at once (continuous batching).
//
// A FIFO queue of requests, a device-memory budget and `max_slots` worker threads.  A slot
// takes the queue head as soon as the head's footprint fits in the unused budget, registers
// the pair (the same Gauss-Newton-Krylov driver as bl_lddmm_register) on the slot's own HIP
// stream in a device arena the slot keeps and reuses, and frees the budget when done, so the
// pairs' kernels overlap on the device and finished pairs are replaced without waiting for
// the others.  Arenas grow to the largest footprint a slot has seen and are otherwise never
// reallocated, so the steady state performs no device allocation.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bl_host.h"

namespace {

using namespace bl::host;
using Clock = std::chrono::steady_clock;

enum ReqState { QUEUED, RUNNING, DONE, CANCELLED };

struct Request {
  uint64_t id = 0;
  bl_problem prob{};
  bl_solver_opts opts{};
  bl::Geo g{};
  size_t bytes = 0;
  std::vector<float> I0, I1, v, warped;
  bl_stats stats{};
  bl_request_times times{};
  int state = QUEUED;
  int rc = BL_OK;
  std::string err;
};

struct Slot {
  std::thread th;
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  double* hscal = nullptr;
  bl_ctx* ctx = nullptr;   // the last request's context (tables built), reused for the same problem
};

}  // namespace

struct bl_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t budget = 0, in_use = 0, peak = 0;
  int resident = 0, peak_resident = 0;
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0;
  int max_slots = 0;
  bool stopping = false;
  uint64_t next_id = 1;
  int device = 0;
  Clock::time_point t0;
  std::vector<Slot> slots;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Run one request on a slot: context in the slot's arena, registration, results to host.
bool same_request_problem(const bl_problem& a, const bl_problem& b) {
  if (a.dim != b.dim || a.nt != b.nt || a.s != b.s || a.gamma != b.gamma ||
      a.precision != b.precision || a.flags != b.flags || a.alpha != b.alpha || a.sigma != b.sigma)
    return false;
  for (int j = 0; j < 3; ++j)
    if (a.n[j] != b.n[j] || a.k[j] != b.k[j]) return false;
  return true;
}

void run_request(bl_server* srv, Slot& slot, int slot_index, Request* r) {
  r->rc = guarded([&]() {
    // a context of the same problem as the slot's last one is reused as it is (its tables
    // and launch shapes); any other problem gets a new context in the slot's arena
    if (slot.ctx && !same_request_problem(slot.ctx->prob, r->prob)) {
      destroy_ctx(slot.ctx);
      slot.ctx = nullptr;
    }
    if (!slot.ctx) {
      if (slot.arena_bytes < r->bytes) {
        if (slot.arena) HIP_TRY(hipFree(slot.arena));
        slot.arena = nullptr;
        slot.arena_bytes = 0;
        HIP_TRY(hipMalloc(&slot.arena, r->bytes));
        slot.arena_bytes = r->bytes;
      }
      slot.ctx = create_ctx(&r->prob, r->g, true, true, slot.arena, slot.arena_bytes, slot.stream,
                            slot.hscal);
    }
    bl_ctx* c = slot.ctx;
    c->have_v = false;
    struct Guard {   // a failed request leaves no context behind
      Slot& sl;
      bool ok = false;
      ~Guard() {
        if (!ok) {
          destroy_ctx(sl.ctx);
          sl.ctx = nullptr;
        }
      }
    } guard{slot};
    load_images(c, r->I0.data(), r->I1.data());
    load_band(c, r->v.data(), c->sv, r->g.nodes * r->g.dim);
    std::memset(&r->stats, 0, sizeof(r->stats));
    const auto ts = Clock::now();
    solve(c, r->opts, &r->stats);
    store_band(c, c->sv, r->v.data(), r->g.nodes * r->g.dim);
    r->warped.resize((size_t)r->g.M);
    store_plane(c, c->mfinal, r->warped.data(), 1);
    sync(c);
    r->stats.seconds = std::chrono::duration<double>(Clock::now() - ts).count();
    guard.ok = true;
    return BL_OK;
  });
  if (r->rc != BL_OK) r->err = bl_lddmm_last_error();
  (void)srv;
  (void)slot_index;
}

void worker(bl_server* srv, int index) {
  Slot& slot = srv->slots[index];
  hipSetDevice(srv->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_work.wait(lk, [&]() {
        if (srv->stopping) return true;
        return !srv->queue.empty() && srv->in_use + srv->queue.front()->bytes <= srv->budget;
      });
      if (srv->stopping) return;
      r = srv->queue.front();
      srv->queue.pop_front();
      r->state = RUNNING;
      r->times.admitted = srv->now();
      r->times.slot = index;
      srv->in_use += r->bytes;
      srv->peak = std::max(srv->peak, srv->in_use);
      srv->resident += 1;
      srv->peak_resident = std::max(srv->peak_resident, srv->resident);
    }
    run_request(srv, slot, index, r);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->in_use -= r->bytes;
      srv->resident -= 1;
      r->times.finished = srv->now();
      r->state = DONE;
      if (r->rc == BL_OK) srv->completed += 1; else srv->failed += 1;
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int bl_server_create(uint64_t budget_bytes, int32_t max_slots, bl_server** out) {
  if (out) *out = nullptr;
  if (!out) return fail(BL_E_INVALID, "NULL pointer argument");
  if (max_slots < 1 || max_slots > 64) return fail(BL_E_INVALID, "max_slots must be in [1, 64]");
  return guarded([&]() {
    std::unique_ptr<bl_server> s(new bl_server());
    HIP_TRY(hipGetDevice(&s->device));
    if (budget_bytes == 0) {
      size_t free_b = 0, total_b = 0;
      HIP_TRY(hipMemGetInfo(&free_b, &total_b));
      budget_bytes = (uint64_t)(0.8 * (double)free_b);
    }
    s->budget = budget_bytes;
    s->max_slots = max_slots;
    s->t0 = Clock::now();
    s->slots.resize(max_slots);
    for (auto& sl : s->slots) {
      HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
      sl.hscal = alloc_host_scalars();
    }
    bl_server* raw = s.get();
    for (int i = 0; i < max_slots; ++i) raw->slots[i].th = std::thread(worker, raw, i);
    *out = s.release();
    return BL_OK;
  });
}

int bl_server_submit(bl_server* srv, const bl_problem* prob, const bl_solver_opts* opts,
                     const float* I0, const float* I1, const float* v_hat, uint64_t* ticket) {
  if (!srv || !I0 || !I1 || !ticket) return fail(BL_E_INVALID, "NULL pointer argument");
  bl::Geo g;
  if (int rc = validate(prob, &g)) return rc;
  if (int rc = validate_opts(opts)) return rc;
  if (prob->flags & BL_DEVICE_PTRS)
    return fail(BL_E_INVALID, "serving takes host pointers (BL_DEVICE_PTRS not allowed)");
  std::unique_ptr<Request> r(new Request());
  r->prob = *prob;
  r->prob.stream = nullptr;
  if (opts) r->opts = *opts; else fill_default(&r->opts);
  r->g = g;
  r->bytes = ctx_bytes(g, true, true, prob->precision == BL_MIXED);
  const size_t M = (size_t)g.M, nb = 2 * (size_t)g.nodes * (size_t)g.dim * (size_t)g.B;
  r->I0.assign(I0, I0 + M);
  r->I1.assign(I1, I1 + M);
  if (v_hat) r->v.assign(v_hat, v_hat + nb); else r->v.assign(nb, 0.f);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (r->bytes > srv->budget) return fail(BL_E_NOMEM, "request footprint exceeds the server budget");
  r->id = srv->next_id++;
  r->times.submitted = srv->now();
  r->times.slot = -1;
  *ticket = r->id;
  srv->queue.push_back(r.get());
  srv->all[r->id] = std::move(r);
  srv->submitted += 1;
  srv->cv_work.notify_all();
  return BL_OK;
}

int bl_server_wait(bl_server* srv, uint64_t ticket, double timeout_s, float* v_hat,
                   float* warped, bl_stats* stats, bl_request_times* times) {
  if (!srv) return fail(BL_E_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(BL_E_INVALID, "unknown ticket");
  Request* r = it->second.get();
  auto ready = [&]() { return r->state == DONE || r->state == CANCELLED; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return BL_PENDING;
  }
  if (times) *times = r->times;
  int rc;
  if (r->state == CANCELLED) {
    rc = fail(BL_E_CANCELLED, "request was cancelled");
  } else if (r->rc != BL_OK) {
    rc = fail(r->rc, r->err);
  } else {
    if (v_hat) std::memcpy(v_hat, r->v.data(), r->v.size() * sizeof(float));
    if (warped) std::memcpy(warped, r->warped.data(), r->warped.size() * sizeof(float));
    if (stats) *stats = r->stats;
    rc = BL_OK;
  }
  srv->all.erase(it);
  return rc;
}

int bl_server_cancel(bl_server* srv, uint64_t ticket) {
  if (!srv) return fail(BL_E_INVALID, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(BL_E_INVALID, "unknown ticket");
  Request* r = it->second.get();
  if (r->state != QUEUED) return fail(BL_E_INVALID, "request is not queued");
  srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), r));
  r->state = CANCELLED;
  r->times.finished = srv->now();
  srv->cancelled += 1;
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
  return BL_OK;
}

int bl_server_info_get(bl_server* srv, bl_server_info* info) {
  if (!srv || !info) return fail(BL_E_INVALID, "NULL pointer argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  info->budget_bytes = srv->budget;
  info->peak_bytes = srv->peak;
  info->max_slots = srv->max_slots;
  info->peak_resident = srv->peak_resident;
  info->submitted = srv->submitted;
  info->completed = srv->completed;
  info->failed = srv->failed;
  info->cancelled = srv->cancelled;
  return BL_OK;
}

void bl_server_destroy(bl_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    for (Request* r : srv->queue) {
      r->state = CANCELLED;
      srv->cancelled += 1;
    }
    srv->queue.clear();
  }
  srv->cv_work.notify_all();
  srv->cv_done.notify_all();
  for (auto& sl : srv->slots)
    if (sl.th.joinable()) sl.th.join();
  hipSetDevice(srv->device);
  for (auto& sl : srv->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    destroy_ctx(sl.ctx);   // does not own the arena, stream or host scalars
    sl.ctx = nullptr;
    if (sl.arena) hipFree(sl.arena);
    if (sl.hscal) hipHostFree(sl.hscal);
    if (sl.stream) hipStreamDestroy(sl.stream);
  }
  delete srv;
}

}  // extern "C"
