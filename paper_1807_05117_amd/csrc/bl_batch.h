// Batched Gauss-Newton-Krylov engine (internal): a cohort of resident registration problems
// of one shape, advanced together one Newton step at a time.
//
// Every problem of a cohort owns one arena of equal layout, `stride` bytes after the previous
// problem's, so one launch of any kernel of the solver path serves all of them (the batch
// descriptor of bl::Geo: grid z = problem, buffers shifted by problem * stride, a per-problem
// gate in device memory).  One Newton step -- the PCG iterations, the slope, one line-search
// trial and, when the trial is accepted, the projected velocity, the gradient and its norms --
// is captured once as a HIP graph and replayed; which problems take part in which part is
// decided on the device by the control kernels from the same FP64 quantities and comparisons
// as the host driver of a single registration (the stopping test of PCG, non-positive
// curvature, the Armijo test), so a problem's result does not depend on its companions.  The
// host reads one control block per problem after each step.
#pragma once

#include <vector>

#include "bl_host.h"

namespace bl {
namespace batch {

// Per-problem control block of a step.  The device copy lives in the problem's scalar area
// (kCtlSlot doubles into bl_ctx::scal); the host copy in pinned, device-mapped memory is
// loaded at the start of a step and stored back at its end, both by kernels of the graph.
struct Ctl {
  // gates: 1 = the problem takes part in that part of the step
  int g_init;    // evaluate the initial velocity: |I0 - I1|^2, state, energy, gradient
  int g_pstart;  // begin PCG: delta = 0, r = -g, z = K r, p = z
  int g_pcg;     // PCG iterations (cleared on the device when PCG stops)
  int g_slope;   // PCG stopped in this step: <g, delta>, eps = 1 follow
  int g_trial;   // a line-search trial at stry = v + eps delta (stays set after a rejection)
  int g_eval;    // state and energy at stry this step (trial or initial velocity)
  int g_grad;    // accepted: projected velocity, gradient, gradient norms
  int g_copyz;   // PCG met non-positive curvature at its first product: delta = z
  // outcomes and counters of the step (the host zeroes hv, evals, grads before each step)
  int iters;     // PCG iterations of the current Newton iteration
  int hv;        // Hessian-vector products in this step
  int trials;    // line-search trials of the current Newton iteration
  int evals;     // state evaluations in this step
  int grads;     // gradients in this step
  int accepted;  // a trial was accepted in this step
  int stalled;   // no trial accepted within max_halvings halvings
  int nonfinite; // non-finite energy or band output
  int max_pcg;
  int max_halvings;
  // FP64 inputs and results
  double thr2;   // PCG stops when max(<r, r>, 0) <= thr2
  double c1;     // Armijo constant
  double sig2M;  // sigma^2 * M (data term of E)
  double eps;    // step length of the next or last trial
  double slope;  // <g, delta>
  double E;      // energy at the current velocity (after acceptance: the accepted one)
  double reg, data;   // regulariser and data sums at the last evaluation
  double gg, ginf;    // <g, g> and max |g| of the last gradient
  double den;         // |I0 - I1|^2
};

constexpr int kMaxPcgPerStep = 10;   // PCG iterations of the largest step graph
// Device bytes the time steps of a cohort's pairs may touch together and still be served by
// the last-level cache between steps (the 256 MiB MALL, minus room for the rest): the offset
// and velocity fields are re-read by every time step, so a cohort larger than this turns
// those cache hits into HBM reads.
constexpr double kLlcBytes = 192.0 * 1024 * 1024;
constexpr int kCtlSlot = 16;   // doubles into bl_ctx::scal (64 doubles, S_SLOTS used before)
static_assert(sizeof(Ctl) <= (64 - kCtlSlot) * sizeof(double), "control block too large");

// Whether a problem can join a cohort: the stationary state equation with Gauss-Newton
// products (gamma 0 or 1), FP32 or mixed precision, host pointers.
bool batchable(const bl_problem& p);

class Cohort {
 public:
  // capacity problems of `prob` (validated into g) on the current device; allocates the arena,
  // the contexts, the stream and the pinned control blocks
  Cohort(const bl_problem& prob, const Geo& g, int capacity);
  ~Cohort();
  Cohort(const Cohort&) = delete;
  Cohort& operator=(const Cohort&) = delete;

  static size_t problem_bytes(const bl_problem& prob, const Geo& g);
  const bl_problem& problem() const { return prob_; }
  int capacity() const { return cap_; }
  size_t bytes() const { return (size_t)cap_ * stride_; }

  // copy a problem's images and initial guess into slot s (stream-ordered, host pointers)
  void load(int s, const float* I0, const float* I1, const float* v);
  // choose launch shapes on slot s's data (once, after the first load); the step graphs are
  // captured at their first launch
  void prepare(int s);
  // pairs whose time-step working set fits the last-level cache together
  static int llc_capacity(const Geo& g);
  Ctl& ctl_in(int s) { return hin_[s]; }
  const Ctl& ctl_out(int s) const { return hout_[s]; }
  // enqueue one step (k_pcg PCG iterations, 0..kMaxPcgPerStep, then the line-search trial and
  // gradient) of every problem whose gates are set in ctl_in; wait or poll for its end
  void launch(int k_pcg);
  void wait();
  bool poll();
  bool in_flight() const { return in_flight_; }
  // results of slot s: velocity (nb floats) and the warped source m(1) (M floats)
  void store(int s, float* v, float* warped);
  // state of the current velocity of slot s (after a stalled line search left a trial's)
  void restore_state(int s);
  hipStream_t stream() const { return stream_; }

 private:
  void enqueue_step(int k_pcg);
  hipGraphExec_t graph(int k_pcg);
  void release();
  Batch gated(const int* gate) const;

  bl_problem prob_{};
  Geo g_{};
  int cap_ = 0;
  size_t stride_ = 0;
  char* arena_ = nullptr;
  hipStream_t stream_ = nullptr;
  std::vector<bl_ctx*> ctx_;
  std::vector<double*> hscal_;
  Ctl* hin_ = nullptr;   // pinned host control blocks (step inputs)
  Ctl* hout_ = nullptr;  // pinned host control blocks (step outputs)
  Ctl* din_ = nullptr;   // their device addresses
  Ctl* dout_ = nullptr;
  std::vector<hipGraphExec_t> exec_;   // step graphs by PCG iterations per step
  bool prepared_ = false;
  hipEvent_t done_ = nullptr;
  bool in_flight_ = false;
};

}  // namespace batch
}  // namespace bl
