// Serving: many registrations resident on one GPU at once (continuous batching).
//
// Two engines behind one request queue and one device-memory budget:
//
// Slot threads (bl_server_create): `max_slots` worker threads.  A free slot takes the queue
// head as soon as the memory it needs fits in the budget, registers the pair (the same
// Gauss-Newton-Krylov driver as bl_lddmm_register) on the slot's own HIP stream in a device
// arena the slot keeps, and takes the next request when done, so the pairs' kernels overlap
// on the device.  The budget is charged with every slot's arena as long as the slot holds it;
// an idle slot frees its arena when the head of the queue needs the memory.
//
// Cohorts (bl_server_create_batched): one scheduler thread.  Requests of equal problems
// (grid, band, Nt, model, precision) share a cohort: up to `max_pairs` resident pairs whose
// device state lies in one arena at a fixed stride, advanced together one Newton step at a
// time by one replay of the cohort's captured step graph (every kernel one launch for all its
// pairs; see bl_batch.h).  New requests join free slots of a cohort between steps; a cohort's
// whole arena is charged to the budget while it exists, and an empty cohort is freed when a
// request of another shape needs the memory.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bl_batch.h"
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
  bool busy = false;
};

// a request resident in a cohort slot, with the host side of its Gauss-Newton loop
struct Resident {
  Request* r = nullptr;
  int phase = 0;         // 0 free, 1 initial evaluation pending, 2 Gauss-Newton iterations
  int it = 0;            // current Gauss-Newton iteration
  bool pcg_open = false; // PCG of iteration `it` runs
  int last_pcg = 0;      // PCG iterations of the previous Gauss-Newton iteration (0: none yet)
  double ginf0 = 0, g0n = 0, gg = 0, ginf = 0;
};

struct CohortEntry {
  std::unique_ptr<bl::batch::Cohort> co;
  std::vector<Resident> res;
  int active = 0;
  bool launched = false;
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
  bool batched = false;
  bool stopping = false;
  std::thread sched;
  std::vector<std::unique_ptr<CohortEntry>> cohorts;   // owned by the scheduler thread
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
    // and launch shapes); any other problem gets a new context in the slot's arena (the
    // worker has sized the arena and charged it to the budget)
    if (slot.ctx && !same_request_problem(slot.ctx->prob, r->prob)) {
      destroy_ctx(slot.ctx);
      slot.ctx = nullptr;
    }
    if (!slot.ctx)
      slot.ctx = create_ctx(&r->prob, r->g, true, true, slot.arena, slot.arena_bytes, slot.stream,
                            slot.hscal);
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

// the slot's context and arena are given back to the device (their bytes leave the budget)
void release_slot_memory(bl_server* srv, Slot& slot) {
  destroy_ctx(slot.ctx);
  slot.ctx = nullptr;
  if (slot.arena) (void)hipFree(slot.arena);
  slot.arena = nullptr;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->in_use -= slot.arena_bytes;
  slot.arena_bytes = 0;
}

void finish_request(bl_server* srv, Request* r) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->resident -= 1;
    r->times.finished = srv->now();
    r->state = DONE;
    if (r->rc == BL_OK) srv->completed += 1; else srv->failed += 1;
  }
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
}

void admit_locked(bl_server* srv, Request* r, int slot_index) {
  r->state = RUNNING;
  r->times.admitted = srv->now();
  r->times.slot = slot_index;
  srv->resident += 1;
  srv->peak_resident = std::max(srv->peak_resident, srv->resident);
}

// Slot thread.  The budget is charged with the slot's arena while the slot holds it: taking
// the head of the queue needs max(arena, footprint) to fit beside every other slot's arena; a
// slot that cannot take the head gives its own arena back, so the head is admitted once
// enough idle memory is returned.
void worker(bl_server* srv, int index) {
  Slot& slot = srv->slots[index];
  (void)hipSetDevice(srv->device);
  for (;;) {
    Request* r = nullptr;
    size_t need = 0;
    bool give_back = false;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      for (;;) {
        if (srv->stopping) return;
        if (!srv->queue.empty()) {
          Request* h = srv->queue.front();
          need = std::max(slot.arena_bytes, h->bytes);
          if (srv->in_use - slot.arena_bytes + need <= srv->budget) {
            r = h;
            srv->queue.pop_front();
            srv->in_use += need - slot.arena_bytes;   // reserved before the allocation
            srv->peak = std::max(srv->peak, srv->in_use);
            admit_locked(srv, r, index);
            break;
          }
          if (slot.arena_bytes > 0) {
            give_back = true;
            break;
          }
        }
        srv->cv_work.wait(lk);
      }
    }
    if (give_back) {
      release_slot_memory(srv, slot);
      srv->cv_work.notify_all();
      continue;
    }
    if (need > slot.arena_bytes) {
      // a larger arena: the old one (and its context) first, then exactly the footprint
      destroy_ctx(slot.ctx);
      slot.ctx = nullptr;
      if (slot.arena) (void)hipFree(slot.arena);
      slot.arena = nullptr;
      if (hipMalloc(&slot.arena, need) != hipSuccess) {
        slot.arena = nullptr;
        {
          std::lock_guard<std::mutex> lk(srv->mu);
          srv->in_use -= need;
          slot.arena_bytes = 0;
        }
        r->rc = BL_E_NOMEM;
        r->err = "device memory for the slot arena is not available";
        finish_request(srv, r);
        continue;
      }
      slot.arena_bytes = need;
    }
    run_request(srv, slot, index, r);
    finish_request(srv, r);
  }
}

// ------------------------------------------------------------------------- cohort scheduler
using bl::batch::Cohort;
using bl::batch::Ctl;

void fail_resident(bl_server* srv, CohortEntry& ce, int s, int rc, const std::string& msg) {
  Resident& R = ce.res[s];
  R.r->rc = rc;
  R.r->err = msg;
  finish_request(srv, R.r);
  R = Resident{};
  ce.co->ctl_in(s) = Ctl{};
  ce.active -= 1;
}

void complete_resident(bl_server* srv, CohortEntry& ce, int s) {
  Resident& R = ce.res[s];
  Request* r = R.r;
  r->rc = guarded([&]() {
    r->warped.resize((size_t)r->g.M);
    ce.co->store(s, r->v.data(), r->warped.data());
    return BL_OK;
  });
  if (r->rc != BL_OK) r->err = bl_lddmm_last_error();
  r->stats.seconds = srv->now() - r->times.admitted;
  finish_request(srv, r);
  R = Resident{};
  ce.co->ctl_in(s) = Ctl{};
  ce.active -= 1;
}

// Begin Gauss-Newton iteration R.it, or end the registration (same tests and order as the
// single-registration driver).  Returns false when the request is complete.
bool begin_iteration(Resident& R, Ctl& in) {
  const bl_solver_opts& o = R.r->opts;
  if (R.it >= o.max_gn) return false;
  if (R.ginf / R.ginf0 < o.gtol) {
    R.r->stats.status = BL_CONVERGED;
    return false;
  }
  const double gn = std::sqrt(std::max(R.gg, 0.0));
  const double eta = std::min(0.5, std::sqrt(gn / R.g0n));
  const double thr = eta * gn;
  in.thr2 = thr * thr;
  in.iters = 0;
  in.g_pstart = 1;
  in.g_pcg = 1;   // max_pcg >= 1
  R.pcg_open = true;
  return true;
}

// Read slot s's control block after a step and prepare its next step.
void advance(bl_server* srv, CohortEntry& ce, int s) {
  Resident& R = ce.res[s];
  Request* r = R.r;
  const Ctl out = ce.co->ctl_out(s);
  Ctl& in = ce.co->ctl_in(s);
  in = out;   // the device's state carries over to the next step
  in.hv = in.evals = in.grads = 0;
  in.accepted = 0;
  in.g_pstart = 0;
  bl_stats& st = r->stats;
  st.hessvecs += out.hv;
  st.evaluations += out.evals;
  if (out.nonfinite) {
    fail_resident(srv, ce, s, BL_E_NONFINITE,
                  out.grads || R.phase == 2 ? "non-finite value in gradient"
                                            : "non-finite value in energy");
    return;
  }
  const bl_solver_opts& o = r->opts;
  auto mse = [&](double data) { return out.den > 0 ? 100.0 * data / out.den : 0.0; };
  if (R.phase == 1) {   // initial velocity evaluated: energy and gradient
    st.E[0] = out.E;
    st.mse_rel[0] = mse(out.data);
    st.ginf_rel[0] = 1.0;
    st.gradients = out.grads;
    st.status = BL_MAXITER;
    if (out.ginf == 0.0) {
      st.status = BL_CONVERGED;
      st.ginf_rel[0] = 0.0;
      complete_resident(srv, ce, s);
      return;
    }
    R.phase = 2;
    R.ginf0 = out.ginf;
    R.g0n = std::sqrt(std::max(out.gg, 0.0));
    R.gg = out.gg;
    R.ginf = out.ginf;
    R.it = 0;
    if (!begin_iteration(R, in)) complete_resident(srv, ce, s);
    return;
  }
  if (R.pcg_open && !out.g_pcg) {
    st.pcg_iters[R.it] = out.iters;
    st.pcg_total += out.iters;
    R.pcg_open = false;
    R.last_pcg = out.iters;
  }
  if (out.accepted) {
    st.ls_trials[R.it] = out.trials;
    st.eps[R.it] = out.eps;
    st.gradients += out.grads;
    st.gn_iters += 1;
    R.gg = out.gg;
    R.ginf = out.ginf;
    st.E[st.gn_iters] = out.E;
    st.mse_rel[st.gn_iters] = mse(out.data);
    st.ginf_rel[st.gn_iters] = R.ginf / R.ginf0;
    if (R.it + 1 == o.max_gn && R.ginf / R.ginf0 < o.gtol) st.status = BL_CONVERGED;
    R.it += 1;
    if (!begin_iteration(R, in)) complete_resident(srv, ce, s);
    return;
  }
  if (out.stalled) {
    st.ls_trials[R.it] = out.trials;
    st.status = BL_STALLED;
    st.eps[R.it] = 0.0;
    const int rc = guarded([&]() {
      ce.co->restore_state(s);   // the state of the returned velocity
      return BL_OK;
    });
    if (rc != BL_OK) fail_resident(srv, ce, s, rc, bl_lddmm_last_error());
    else complete_resident(srv, ce, s);
  }
  // otherwise PCG continues or the line search retries with half the step in the next step
}

// Admit queued requests into cohort slots (FIFO; a request joins a free slot of a cohort of
// its problem or a new cohort; empty cohorts of other problems are freed when the memory is
// needed).  Cohorts are created and loaded outside the lock.
void admit_batched(bl_server* srv, int max_pairs) {
  struct Plan {
    Request* r;
    CohortEntry* ce;   // null: the new cohort `fresh`
    int fresh;
  };
  struct Fresh {
    bl_problem prob;
    bl::Geo g;
    int cap;
    std::unique_ptr<CohortEntry> ce;
  };
  std::vector<Plan> plan;
  std::vector<Fresh> fresh;
  std::vector<std::unique_ptr<CohortEntry>> drop;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return;
    std::vector<int> used(srv->cohorts.size(), 0);
    std::vector<int> fresh_used;
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
      Request* r = *it;
      // at most max_pairs pairs resident over all cohorts
      if (srv->resident >= max_pairs) break;
      bool placed = false, defer = false;
      if (bl::batch::batchable(r->prob)) {
        for (size_t i = 0; i < srv->cohorts.size() && !placed; ++i) {
          CohortEntry& ce = *srv->cohorts[i];
          if (!ce.co || !same_request_problem(ce.co->problem(), r->prob)) continue;
          if (ce.active + used[i] < ce.co->capacity()) {
            // a cohort in flight reads its control blocks: it takes requests after its step
            if (ce.launched) {
              defer = true;
              continue;
            }
            plan.push_back({r, &ce, -1});
            used[i] += 1;
            placed = true;
          }
        }
        if (!placed && defer) {
          if (it == srv->queue.begin()) break;
          ++it;
          continue;
        }
        for (size_t f = 0; f < fresh.size() && !placed; ++f) {
          if (same_request_problem(fresh[f].prob, r->prob) && fresh_used[f] < fresh[f].cap) {
            plan.push_back({r, nullptr, (int)f});
            fresh_used[f] += 1;
            placed = true;
          }
        }
        if (!placed) {
          // a new cohort: free empty cohorts of other problems while the memory is short
          for (size_t i = 0; i < srv->cohorts.size() && srv->in_use + r->bytes > srv->budget;
               ++i) {
            CohortEntry& ce = *srv->cohorts[i];
            if (ce.co && ce.active == 0 && used[i] == 0 && !ce.launched) {
              srv->in_use -= ce.co->bytes();
              drop.push_back(std::move(srv->cohorts[i]));
              srv->cohorts[i].reset(new CohortEntry());   // placeholder, removed below
            }
          }
          const uint64_t room = srv->budget - std::min(srv->budget, srv->in_use);
          const int cap = (int)std::min<uint64_t>(
              (uint64_t)std::min(max_pairs, Cohort::llc_capacity(r->g)), room / r->bytes);
          if (cap >= 1) {
            Fresh f{r->prob, r->g, cap, nullptr};
            fresh.push_back(std::move(f));
            fresh_used.push_back(1);
            srv->in_use += (uint64_t)cap * r->bytes;
            srv->peak = std::max(srv->peak, srv->in_use);
            plan.push_back({r, nullptr, (int)fresh.size() - 1});
            placed = true;
          }
        }
      } else {
        // other models are not batched: the request fails at once
        r->rc = BL_E_UNSUPPORTED;
        r->err = "the cohort server registers the stationary Gauss-Newton state-equation model "
                 "(BL_NEWTON, BL_NONSTATIONARY and BL_DEFORMATION need bl_server_create)";
        r->state = DONE;
        r->times.admitted = r->times.finished = srv->now();
        srv->failed += 1;
        it = srv->queue.erase(it);
        srv->cv_done.notify_all();
        continue;
      }
      if (!placed) {
        if (it == srv->queue.begin()) break;   // the head waits for memory; FIFO order kept
        ++it;
        continue;
      }
      admit_locked(srv, r, -1);
      it = srv->queue.erase(it);
    }
    // remove the placeholders of freed cohorts
    srv->cohorts.erase(std::remove_if(srv->cohorts.begin(), srv->cohorts.end(),
                                      [](const std::unique_ptr<CohortEntry>& e) { return !e->co; }),
                       srv->cohorts.end());
  }
  drop.clear();   // frees the empty cohorts' memory (outside the lock)
  // create the new cohorts
  for (Fresh& f : fresh) {
    f.ce.reset(new CohortEntry());
    const int rc = guarded([&]() {
      f.ce->co.reset(new Cohort(f.prob, f.g, f.cap));
      return BL_OK;
    });
    if (rc != BL_OK) f.ce.reset();
    f.ce ? (void)f.ce->res.resize(f.cap) : (void)0;
  }
  // load the admitted requests
  std::vector<CohortEntry*> fresh_ptrs(fresh.size(), nullptr);
  for (size_t f = 0; f < fresh.size(); ++f) {
    if (!fresh[f].ce) {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->in_use -= (uint64_t)fresh[f].cap * Cohort::problem_bytes(fresh[f].prob, fresh[f].g);
      continue;
    }
    fresh_ptrs[f] = fresh[f].ce.get();
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->cohorts.push_back(std::move(fresh[f].ce));
  }
  for (const Plan& pl : plan) {
    CohortEntry* ce = pl.ce ? pl.ce : fresh_ptrs[pl.fresh];
    Request* r = pl.r;
    if (!ce) {
      r->rc = BL_E_NOMEM;
      r->err = "device memory for a new cohort is not available";
      finish_request(srv, r);
      continue;
    }
    int s = 0;
    while (ce->res[s].r) ++s;
    Resident& R = ce->res[s];
    R = Resident{};
    R.r = r;
    R.phase = 1;
    std::memset(&r->stats, 0, sizeof(r->stats));
    r->times.slot = s;
    const int rc = guarded([&]() {
      ce->co->load(s, r->I0.data(), r->I1.data(), r->v.data());
      ce->co->prepare(s);
      return BL_OK;
    });
    ce->active += 1;
    Ctl& in = ce->co->ctl_in(s);
    in = Ctl{};
    if (rc != BL_OK) {
      fail_resident(srv, *ce, s, rc, bl_lddmm_last_error());
      continue;
    }
    const double sig = r->prob.sigma;
    in.g_init = 1;
    in.c1 = r->opts.c1;
    in.sig2M = sig * sig * (double)r->g.M;
    in.max_pcg = r->opts.max_pcg;
    in.max_halvings = r->opts.max_halvings;
  }
}

// PCG iterations of a cohort's next step: enough for the pair expected to need the most
// (each pair's previous Gauss-Newton iteration's count, at least one more), so that few
// gated-off iterations run; 0 when no pair is in PCG (initial evaluations, line-search
// retries).  BL_COHORT_PCG_PER_STEP fixes the number instead.
int pcg_per_step(const CohortEntry& ce) {
  static const int fixed = []() {
    const char* e = std::getenv("BL_COHORT_PCG_PER_STEP");
    return e ? std::atoi(e) : -1;
  }();
  int k = 0;
  for (size_t s = 0; s < ce.res.size(); ++s) {
    const Resident& R = ce.res[s];
    if (!R.r || R.phase != 2 || !R.pcg_open) continue;
    const Ctl& in = ce.co->ctl_in((int)s);
    const int left = in.max_pcg - in.iters;
    const int guess = std::max(1, (R.last_pcg > 0 ? R.last_pcg : 2) - in.iters);
    k = std::max(k, std::min(left, guess));
  }
  if (k > 0 && fixed >= 1) k = fixed;
  return std::min(k, bl::batch::kMaxPcgPerStep);
}

void scheduler(bl_server* srv, int max_pairs) {
  (void)hipSetDevice(srv->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      bool any = false;
      for (auto& ce : srv->cohorts) any = any || ce->active > 0;
      if (srv->stopping && !any) return;
      if (!any && srv->queue.empty()) {
        srv->cv_work.wait(lk, [&]() { return srv->stopping || !srv->queue.empty(); });
        continue;
      }
    }
    admit_batched(srv, max_pairs);
    bool in_flight = false;
    for (auto& up : srv->cohorts) {
      CohortEntry& ce = *up;
      if (ce.active == 0 || ce.launched) {
        in_flight = in_flight || ce.launched;
        continue;
      }
      const int rc = guarded([&]() {
        ce.co->launch(pcg_per_step(ce));
        return BL_OK;
      });
      if (rc != BL_OK) {
        const std::string msg = bl_lddmm_last_error();
        for (int s = 0; s < (int)ce.res.size(); ++s)
          if (ce.res[s].r) fail_resident(srv, ce, s, rc, msg);
        continue;
      }
      ce.launched = true;
      in_flight = true;
    }
    if (!in_flight) continue;
    // the cohorts whose steps have ended, in any order
    bool progressed = false;
    for (auto& up : srv->cohorts) {
      CohortEntry& ce = *up;
      if (!ce.launched) continue;
      bool ended = false;
      const int rc = guarded([&]() {
        ended = ce.co->poll();
        return BL_OK;
      });
      if (rc == BL_OK && !ended) continue;
      ce.launched = false;
      progressed = true;
      for (int s = 0; s < (int)ce.res.size(); ++s) {
        if (!ce.res[s].r) continue;
        if (rc != BL_OK) fail_resident(srv, ce, s, rc, bl_lddmm_last_error());
        else advance(srv, ce, s);
      }
    }
    if (!progressed) std::this_thread::yield();
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

int bl_server_create_batched(uint64_t budget_bytes, int32_t max_pairs, bl_server** out) {
  if (out) *out = nullptr;
  if (!out) return fail(BL_E_INVALID, "NULL pointer argument");
  if (max_pairs < 1 || max_pairs > 64) return fail(BL_E_INVALID, "max_pairs must be in [1, 64]");
  return guarded([&]() {
    std::unique_ptr<bl_server> s(new bl_server());
    HIP_TRY(hipGetDevice(&s->device));
    if (budget_bytes == 0) {
      size_t free_b = 0, total_b = 0;
      HIP_TRY(hipMemGetInfo(&free_b, &total_b));
      budget_bytes = (uint64_t)(0.8 * (double)free_b);
    }
    s->budget = budget_bytes;
    s->max_slots = max_pairs;
    s->batched = true;
    s->t0 = Clock::now();
    bl_server* raw = s.get();
    raw->sched = std::thread(scheduler, raw, max_pairs);
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
  if (srv->sched.joinable()) srv->sched.join();
  (void)hipSetDevice(srv->device);
  srv->cohorts.clear();
  for (auto& sl : srv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    destroy_ctx(sl.ctx);   // does not own the arena, stream or host scalars
    sl.ctx = nullptr;
    if (sl.arena) (void)hipFree(sl.arena);
    if (sl.hscal) (void)hipHostFree(sl.hscal);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete srv;
}

}  // extern "C"
