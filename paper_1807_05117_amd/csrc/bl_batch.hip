// Batched Gauss-Newton-Krylov engine: cohorts of resident problems of one shape, one fused
// multi-problem launch per kernel of the solver path, each Newton step replayed from a
// captured HIP graph with the solver's decisions taken per problem on the device.
//
// The step follows the reduced-space Gauss-Newton-Krylov iteration of the paper (Section 3.4,
// equations BLNewton and BLKKT; PCG preconditioned by K~ = L~^-1, Armijo backtracking on E)
// in the same order and FP64 arithmetic as the host driver of one registration:
//   PCG:    delta = 0, r = -g, z = K r, p = z;  per iteration Hp, <p, Hp>, the PCG update, and
//           stop on <p, Hp> <= 0 (delta = z if that happens at the first product), on
//           max(<r, r>, 0) <= (eta |g|)^2, or after max_pcg iterations
//   slope:  <g, delta>, eps = 1
//   trial:  v + eps delta, state and E; accept if E <= E_0 + c1 eps slope, else halve eps
//           (the next step retries) until max_halvings halvings
//   accept: v <- projected trial, gradient, <g, g>, max |g|
// The control kernels evaluate these tests with floating-point contraction disabled, so each
// FP64 operation rounds exactly as the host's does.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "bl_batch.h"

namespace bl {
namespace batch {
namespace {

using namespace bl::host;

__device__ __forceinline__ Ctl* ctl_of(char* scal0, int64_t stride, int p) {
  return reinterpret_cast<Ctl*>(scal0 + (int64_t)p * stride + kCtlSlot * sizeof(double));
}
__device__ __forceinline__ double* scal_of(char* scal0, int64_t stride, int p) {
  return reinterpret_cast<double*>(scal0 + (int64_t)p * stride);
}

// step inputs from the pinned host blocks into the problems' scalar areas
__global__ __launch_bounds__(64) void k_ctl_load(const Ctl* __restrict__ src, char* scal0,
                                                 int64_t stride, int count) {
  const int p = threadIdx.x;
  if (p < count) *ctl_of(scal0, stride, p) = src[p];
}

__global__ __launch_bounds__(64) void k_ctl_store(Ctl* __restrict__ dst, char* scal0,
                                                  int64_t stride, int count) {
  const int p = threadIdx.x;
  if (p < count) dst[p] = *ctl_of(scal0, stride, p);
}

// after the PCG update of one iteration: count the product, stop on non-positive curvature,
// on the forcing test or at max_pcg
__global__ __launch_bounds__(64) void k_ctl_pcg(char* scal0, int64_t stride, int count) {
#pragma clang fp contract(off)
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  if (!c->g_pcg) return;
  const double* sc = scal_of(scal0, stride, p);
  c->hv += 1;
  const double php = sc[S_PHP];
  bool stop = false;
  if (!(php > 0.0)) {
    if (c->iters == 0) c->g_copyz = 1;   // the preconditioned steepest-descent step
    stop = true;
  } else {
    c->iters += 1;
    const double rr = sc[S_RR];
    const double rr0 = rr < 0.0 ? 0.0 : rr;   // std::max(rr, 0.0)
    if (rr0 <= c->thr2 || c->iters >= c->max_pcg) stop = true;
  }
  if (stop) {
    c->g_pcg = 0;
    c->g_slope = 1;
  }
}

// problems still in PCG: <r, z> of this iteration becomes the next one's denominator
__global__ __launch_bounds__(64) void k_ctl_swap(char* scal0, int64_t stride, int count) {
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  if (!c->g_pcg) return;
  double* sc = scal_of(scal0, stride, p);
  sc[S_RZ0] = sc[S_RZ1];
}

// PCG stopped in this step: the slope of the line search, the first trial at eps = 1
__global__ __launch_bounds__(64) void k_ctl_slope(char* scal0, int64_t stride, int count) {
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  if (!c->g_slope) return;
  c->slope = scal_of(scal0, stride, p)[S_SLOPE];
  c->eps = 1.0;
  c->trials = 0;
  c->g_slope = 0;
  c->g_copyz = 0;
  c->g_trial = 1;
}

__global__ __launch_bounds__(64) void k_ctl_eval(char* scal0, int64_t stride, int count) {
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  c->g_eval = (c->g_trial || c->g_init) ? 1 : 0;
}

// after the state and energy sums at stry: E, then acceptance (the initial velocity is always
// taken), or a halving of eps, or the end of the line search
__global__ __launch_bounds__(64) void k_ctl_armijo(char* scal0, int64_t stride, int count) {
#pragma clang fp contract(off)
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  if (!c->g_eval) return;
  c->g_eval = 0;
  const double* sc = scal_of(scal0, stride, p);
  const double reg = sc[S_REG], data = sc[S_DATA];
  const double E = 0.5 * reg + data / c->sig2M;
  c->evals += 1;
  if (c->g_init) c->den = sc[S_SQD];
  if (!isfinite(E)) {
    c->nonfinite = 1;
    c->g_init = 0;
    c->g_trial = 0;
    return;
  }
  bool take = false;
  if (c->g_init) {
    take = true;
    c->g_init = 0;
  } else {
    c->trials += 1;
    if (E <= c->E + c->c1 * c->eps * c->slope) {
      take = true;
      c->accepted = 1;
    } else {
      c->eps *= 0.5;
      if (c->trials >= c->max_halvings + 1) {
        c->stalled = 1;
        c->g_trial = 0;
      }
    }
  }
  if (take) {
    c->g_trial = 0;
    c->g_grad = 1;
    c->E = E;
    c->reg = reg;
    c->data = data;
  }
}

// after the gradient norms: publish them, and the non-finite flag of the band kernels
__global__ __launch_bounds__(64) void k_ctl_grad(char* scal0, int64_t stride, int count,
                                                 char* flag0) {
  const int p = threadIdx.x;
  if (p >= count) return;
  Ctl* c = ctl_of(scal0, stride, p);
  if (!c->g_grad) return;
  c->g_grad = 0;
  const double* sc = scal_of(scal0, stride, p);
  c->gg = sc[S_GG];
  c->ginf = sc[S_GINF];
  c->grads += 1;
  int* flag = reinterpret_cast<int*>(flag0 + (int64_t)p * stride);
  if (*flag) {
    c->nonfinite = 1;
    *flag = 0;
  }
}

}  // namespace

bool batchable(const bl_problem& p) {
  return (p.flags & (BL_DEVICE_PTRS | BL_NEWTON | BL_NONSTATIONARY | BL_DEFORMATION)) == 0 &&
         (p.precision == BL_FP32 || p.precision == BL_MIXED);
}

size_t Cohort::problem_bytes(const bl_problem& prob, const Geo& g) {
  return ctx_bytes(g, true, true, prob.precision == BL_MIXED);
}

Cohort::Cohort(const bl_problem& prob, const Geo& g, int capacity)
    : prob_(prob), g_(g), cap_(capacity) {
  if (cap_ < 1 || cap_ > 64) throw DeviceError{hipErrorInvalidValue, "cohort capacity"};
  prob_.stream = nullptr;
  stride_ = problem_bytes(prob_, g_);   // a multiple of 256 (every buffer is 256-aligned)
  try {
    HIP_TRY(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
    HIP_TRY(hipMalloc((void**)&arena_, (size_t)cap_ * stride_));
    HIP_TRY(hipHostMalloc((void**)&hin_, cap_ * sizeof(Ctl), hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostMalloc((void**)&hout_, cap_ * sizeof(Ctl), hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(hin_, 0, cap_ * sizeof(Ctl));
    std::memset(hout_, 0, cap_ * sizeof(Ctl));
    HIP_TRY(hipHostGetDevicePointer((void**)&din_, hin_, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&dout_, hout_, 0));
    for (int p = 0; p < cap_; ++p) {
      hscal_.push_back(alloc_host_scalars());
      ctx_.push_back(create_ctx(&prob_, g_, true, true, arena_ + (size_t)p * stride_, stride_,
                                stream_, hscal_.back()));
    }
  } catch (...) {
    release();
    throw;
  }
}

Cohort::~Cohort() { release(); }

void Cohort::release() {
  if (stream_) (void)hipStreamSynchronize(stream_);
  for (hipGraphExec_t& e : exec_)
    if (e) (void)hipGraphExecDestroy(e);
  exec_.clear();
  for (bl_ctx* c : ctx_) destroy_ctx(c);   // does not own the arena, stream or host scalars
  ctx_.clear();
  for (double* h : hscal_) (void)hipHostFree(h);
  hscal_.clear();
  if (hin_) (void)hipHostFree(hin_);
  if (hout_) (void)hipHostFree(hout_);
  hin_ = hout_ = nullptr;
  if (arena_) (void)hipFree(arena_);
  arena_ = nullptr;
  if (done_) (void)hipEventDestroy(done_);
  done_ = nullptr;
  if (stream_) (void)hipStreamDestroy(stream_);
  stream_ = nullptr;
}

void Cohort::load(int s, const float* I0, const float* I1, const float* v) {
  bl_ctx* c = ctx_[s];
  load_images(c, I0, I1);
  load_band(c, v, c->sv, g_.dim);
  check_launch("cohort load");
}

void Cohort::prepare(int s) {
  if (prepared_) return;
  // launch shapes from a real state evaluation of the first problem (the tuner times the
  // transports on its offsets; the step graph re-evaluates this problem from scratch)
  bl_ctx* c0 = ctx_[s];
  op_set_velocity(c0, c0->sv);
  for (bl_ctx* c : ctx_) {
    for (int k = 0; k < bl::TR_CLASSES; ++k) c->g.zv[k] = c0->g.zv[k];
    c->tuned = true;
  }
  for (int k = 0; k < bl::TR_CLASSES; ++k) g_.zv[k] = c0->g.zv[k];
  exec_.assign(kMaxPcgPerStep + 1, nullptr);
  prepared_ = true;
}

// the step graph with k PCG iterations, captured at its first use
hipGraphExec_t Cohort::graph(int k) {
  if (exec_[k]) return exec_[k];
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_step(k);
  } catch (...) {
    (void)hipStreamEndCapture(stream_, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIP_TRY(hipStreamEndCapture(stream_, &graph));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw DeviceError{e, "hipGraphInstantiate (cohort step)"};
  exec_[k] = ex;
  return ex;
}

Batch Cohort::gated(const int* gate) const {
  Batch b;
  b.stride = (int64_t)stride_;
  b.gate = gate;
  b.gate_stride = (int64_t)(stride_ / sizeof(int));
  b.count = cap_;
  return b;
}

// The launch sequence of one step on problem 0's buffers; every launch is batched over the
// cohort and gated per problem.  Only kernels (no memset or copy nodes) are captured.
void Cohort::enqueue_step(int k_pcg) {
  bl_ctx* c = ctx_[0];
  hipStream_t s = stream_;
  const Geo g0 = c->g;
  const int64_t nb = (int64_t)g0.dim * g0.B;
  char* scal0 = reinterpret_cast<char*>(c->scal);
  const Ctl* ctl0 = reinterpret_cast<const Ctl*>(scal0 + kCtlSlot * sizeof(double));
  const int64_t st = (int64_t)stride_;
  double* pa = c->red + RED_A * bl::kRedBlocks;
  double* pb = c->red + RED_B * bl::kRedBlocks;
  double* pc = c->red + RED_C * bl::kRedBlocks;
  auto use = [&](const int* gate) {
    c->g = g0;
    c->g.bat = gated(gate);
    return c->g.bat;
  };
  const dim3 one(1), lanes(64);

  hipLaunchKernelGGL(k_ctl_load, one, lanes, 0, s, din_, scal0, st, cap_);

  // initial velocity: stry = v, |I0 - I1|^2
  Batch b = use(&ctl0->g_init);
  bl::copy_band(c->stry, c->sv, nb, s, b);
  bl::sqdiff_partial(c->m, c->I1, g0.M, pa, s, b);
  bl::reduce_final(pa, bl::kRedBlocks, c->scal + S_SQD, s, nullptr, nullptr, nullptr, b);

  // PCG start: delta = 0, r = -g, z = K r with <r, r> and <r, z>, p = z
  b = use(&ctl0->g_pstart);
  bl::zero_band(c->sdelta, nb, s, b);
  bl::zero_band(c->sr, nb, s, b);
  bl::axpy(c->sr, c->sg, -1.0, nb, s, b);
  bl::precond_dots(c->g, c->sr, c->Lhat, c->sz, pa, pb, s);
  bl::reduce_final2(pa, c->scal + S_RR, nullptr, pb, c->scal + S_RZ0, nullptr, bl::kRedBlocks, s,
                    false, nullptr, nullptr, b);
  bl::copy_band(c->sp, c->sz, nb, s, b);

  // PCG iterations
  for (int j = 0; j < k_pcg; ++j) {
    b = use(&ctl0->g_pcg);
    const bool fused = op_hessvec(c, c->sp, c->sHp, pc);
    if (!fused) vec_dot_partial(c, c->sp, c->sHp, pc);
    bl::pcg_step(c->g, c->sp, c->sHp, c->scal + S_RZ0, pc,
                 fused ? bl::finalize_blocks(c->g) : bl::kRedBlocks, c->scal + S_PHP, nullptr,
                 c->sdelta, c->sr, c->Lhat, c->sz, pa, pb, s);
    bl::reduce_final2(pa, c->scal + S_RR, nullptr, pb, c->scal + S_RZ1, nullptr, bl::kRedBlocks,
                      s, false, nullptr, nullptr, b);
    hipLaunchKernelGGL(k_ctl_pcg, one, lanes, 0, s, scal0, st, cap_);
    bl::xpby_dev(c->sp, c->sz, c->scal + S_RZ1, c->scal + S_RZ0, nb, s, b);
    hipLaunchKernelGGL(k_ctl_swap, one, lanes, 0, s, scal0, st, cap_);
  }
  b = use(&ctl0->g_copyz);
  bl::copy_band(c->sdelta, c->sz, nb, s, b);

  // slope of the line search
  b = use(&ctl0->g_slope);
  vec_dot_partial(c, c->sg, c->sdelta, pa);
  bl::reduce_final(pa, bl::kRedBlocks, c->scal + S_SLOPE, s, nullptr, nullptr, nullptr, b);
  hipLaunchKernelGGL(k_ctl_slope, one, lanes, 0, s, scal0, st, cap_);

  // one trial (or the initial velocity): state and energy, Armijo
  hipLaunchKernelGGL(k_ctl_eval, one, lanes, 0, s, scal0, st, cap_);
  b = use(&ctl0->g_trial);
  bl::add_scaled_dev(c->stry, c->sv, c->sdelta, &ctl0->eps, nb, s, b);
  b = use(&ctl0->g_eval);
  enqueue_set_velocity(c, c->stry);
  hipLaunchKernelGGL(k_ctl_armijo, one, lanes, 0, s, scal0, st, cap_);

  // accepted: v = projected trial, gradient and its norms
  b = use(&ctl0->g_grad);
  bl::copy_band(c->sv, c->bv, nb, s, b);
  const bool norms = op_gradient(c, c->sg, pa, pb);   // with the partials of its norms
  if (!norms) {
    vec_dot_partial(c, c->sg, c->sg, pa);
    bl::maxabs_partial(c->sg, nb, pb, s, b);
  }
  bl::reduce_final2(pa, c->scal + S_GG, nullptr, pb, c->scal + S_GINF, nullptr,
                    norms ? bl::finalize_blocks(c->g) : bl::kRedBlocks, s, true, nullptr, nullptr,
                    b);
  hipLaunchKernelGGL(k_ctl_grad, one, lanes, 0, s, scal0, st, cap_,
                     reinterpret_cast<char*>(c->flag));

  hipLaunchKernelGGL(k_ctl_store, one, lanes, 0, s, dout_, scal0, st, cap_);
  c->g = g0;   // problem 0's context is a plain single-problem context again
  check_launch("cohort step");
}

void Cohort::launch(int k_pcg) {
  k_pcg = std::max(0, std::min(k_pcg, kMaxPcgPerStep));
  HIP_TRY(hipGraphLaunch(graph(k_pcg), stream_));
  HIP_TRY(hipEventRecord(done_, stream_));
  in_flight_ = true;
}

void Cohort::wait() {
  if (!in_flight_) return;
  HIP_TRY(hipEventSynchronize(done_));
  in_flight_ = false;
}

bool Cohort::poll() {
  if (!in_flight_) return true;
  const hipError_t e = hipEventQuery(done_);
  if (e == hipErrorNotReady) return false;
  if (e != hipSuccess) throw DeviceError{e, "hipEventQuery (cohort step)"};
  in_flight_ = false;
  return true;
}

int Cohort::llc_capacity(const Geo& g) {
  // grid bytes one incremental-state step of a pair touches: X (dim planes), dv (dim),
  // m^{n+1}, t^n and t^{n+1}
  const double step = (double)g.M * 4.0 * (2.0 * g.dim + 3.0);
  double llc = kLlcBytes;
  if (const char* e = std::getenv("BL_COHORT_LLC_BYTES")) llc = std::atof(e);
  return std::max(1, (int)(llc / step));
}

void Cohort::store(int s, float* v, float* warped) {
  bl_ctx* c = ctx_[s];
  store_band(c, c->sv, v, g_.dim);
  if (warped) store_plane(c, c->mfinal, warped, 1);
  sync(c);
}

void Cohort::restore_state(int s) { op_set_velocity(ctx_[s], ctx_[s]->sv); }

}  // namespace batch
}  // namespace bl
