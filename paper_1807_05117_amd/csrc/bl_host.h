// Host-side internals shared by the C-interface translation units: the device context of one
// registration problem, validation, transfers and the Gauss-Newton-Krylov driver.
#pragma once

#include <string>
#include <vector>

#include "bl_internal.h"
#include "bl_lddmm.h"

namespace bl {
namespace host {

struct DeviceError {
  hipError_t e;
  const char* where;
};

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) throw DeviceError{e_, #expr}; \
  } while (0)

inline void check_launch(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw DeviceError{e, where};
}

struct NonFinite {
  const char* what;
};

enum { RED_REG = 0, RED_DATA, RED_A, RED_B, RED_C, RED_SLOTS };
// slots of the device scalars (bl_ctx::scal) and of their host-mapped mirror (bl_ctx::hscal)
enum {
  S_REG = 0, S_DATA, S_GG, S_GINF, S_PHP, S_SLOPE, S_RR, S_RZ0, S_RZ1, S_SQD, S_FLAG, S_SLOTS
};

int fail(int code, const std::string& msg);
int validate(const bl_problem* p, Geo* g);
int validate_opts(const bl_solver_opts* o);
void fill_default(bl_solver_opts* o);

}  // namespace host
}  // namespace bl

struct bl_ctx {
  bl::Geo g{};
  bl_problem prob{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool devptr = false;
  bool transport = true;
  char* arena = nullptr;
  bool own_arena = true;
  size_t arena_bytes = 0;
  // grid fields
  float* I1 = nullptr;
  float* m = nullptr;      // (nt + 1) planes, m[0] = I0
  float* X = nullptr;      // dim planes: forward departure offsets
  float4* YA = nullptr;    // (Y, a): backward offsets and adjoint reaction factor
  float* V = nullptr;      // dim + 1 planes: v, r (per time node when non-stationary)
  float* DV = nullptr;     // dim planes: dv (per time node when non-stationary)
  float* T0 = nullptr;
  float* T1 = nullptr;
  float* L = nullptr;      // (nt + 1) planes: adjoint or incremental adjoint
  float* Bf = nullptr;     // dim planes: body force (per time node when non-stationary)
  // full Newton products only
  float* DM = nullptr;     // (nt + 1) planes: dm^n (dm^0 = 0)
  float* DL = nullptr;     // (nt + 1) planes: dlambda^n
  float* U0 = nullptr;     // u ping-pong of the incremental adjoint
  float* U1 = nullptr;
  float* mfinal = nullptr;  // m(1): the warped source
  // deformation state equation only (image grid)
  float4* IG = nullptr;    // (I0, central-difference gradient of I0)
  float4* GP = nullptr;    // (grad I0) o phi(1) (w unused)
  float* UG = nullptr;     // dim planes: iota(u~(1)), then iota(du~(1)) in products
  // deformation state equation only (product grid of the truncated convolutions)
  bl::Geo gP{};            // the product grid as a transform geometry
  bl::DftPlan planP;
  bool fused = false;      // the fused stage kernels run the product-grid sweeps
  float* VP = nullptr;     // dim planes: iota(v~)
  float* DVP = nullptr;    // dim planes: iota(dv~)
  float* DUG = nullptr;    // 4 nt stages x dim^2 planes: iota(d~_j U_i) of every stage state
  float* GW = nullptr;     // dim^2 planes of work
  float* KG = nullptr;     // dim planes of work
  float* GACC = nullptr;   // dim planes: deformation part of the gradient integrand
  float2* DUb = nullptr;   // dim^2 band fields: spectral derivatives of a stage state
  float2* US = nullptr;    // 2 x dim band fields: u~_n ping-pong
  float2* ACC = nullptr;   // dim: Runge-Kutta slope sum
  float2* KAP = nullptr;   // dim: transposed-sweep stage cotangent
  float2* RHO = nullptr;   // dim: band adjoint
  float2* ASUM = nullptr;  // dim: running sum of A kap_s within a step
  float2* KSUM = nullptr;  // dim: identity part of the gradient integrand
  float2* PH = nullptr;    // dim^2 half spectra of the product grid
  // band vectors (complex)
  float2* braw = nullptr;  // up to 4 components of staging
  float2* bv = nullptr;    // dim + 1: projected v, divergence
  float2* bd = nullptr;    // dim: projected dv
  float2* bout = nullptr;  // dim
  float2* P = nullptr;     // C_max * kzh * ky * kx half spectra
  float* Lhat = nullptr;
  double* Lhat64 = nullptr;
  bl::DftPlan plan;
  double* red = nullptr;   // RED_SLOTS * kRedBlocks partials
  double* scal = nullptr;  // device scalars
  double* hscal = nullptr; // pinned, coherent host scalars (64 doubles) written by kernels
  double* hdev = nullptr;  // device address of hscal
  bool own_hscal = true;
  int* flag = nullptr;
  double* hflag_dummy = nullptr;
  // transport launch shapes chosen for this grid shape (Geo::zv)
  bool tuned = false;
  // state of the last velocity
  bool have_v = false;
  bool have_lambda = false;   // L holds the adjoint lambda^n of the current velocity
  bool lamT_valid = false;    // L[nt] holds lambda^Nt of the current velocity (with the energy)
  double E = 0, reg = 0, data_sum = 0;
  // solver vectors (dim * B complex each)
  float2 *sv = nullptr, *sg = nullptr, *sdelta = nullptr, *sr = nullptr, *sz = nullptr,
         *sp = nullptr, *sHp = nullptr, *stry = nullptr;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<bl::LaunchEvents> ev_pairs;   // event pairs armed for single launches
  struct Run { int cls, ev, count; };
  std::vector<Run> ev_used;  // timed runs: class, pool index of the start event, launches
  size_t ev_next = 0;

  int64_t t_launch[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double t_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace bl {
namespace host {

// Device bytes of a context (transport fields, solver vectors, mixed-precision tables).
size_t ctx_bytes(const Geo& g, bool transport, bool solver, bool mixed);
// A context on the current device.  With arena != nullptr the caller provides (and keeps
// owning) at least ctx_bytes() of device memory and the stream, and host_scalars (64 doubles
// from alloc_host_scalars) if not NULL; no device memory is allocated then.  host_mirror =
// false: no host-mapped scalars at all (hscal = hdev = NULL, nothing published to the host;
// only operation sequences that read no published scalar may run on such a context).
bl_ctx* create_ctx(const bl_problem* prob, const Geo& g, bool transport, bool solver,
                   void* arena = nullptr, size_t arena_bytes = 0, hipStream_t stream = nullptr,
                   double* host_scalars = nullptr, bool host_mirror = true);
void destroy_ctx(bl_ctx* c);
// owns a context until the end of a scope
struct CtxHolder {
  bl_ctx* c = nullptr;
  ~CtxHolder() { destroy_ctx(c); }
};
// 64 doubles of pinned, coherent, device-mapped host memory for published scalars
double* alloc_host_scalars();
void sync(bl_ctx* c);
void load_images(bl_ctx* c, const float* I0, const float* I1);
void load_band(bl_ctx* c, const float* src, float2* dst, int ncomp);
void store_band(bl_ctx* c, const float2* src, float* dst, int ncomp);
void store_plane(bl_ctx* c, const float* src, float* dst, size_t nplanes);
void solve(bl_ctx* c, const bl_solver_opts& o, bl_stats* st);
// operator sequences on a context (enqueued on c->stream; launches follow c->g.bat)
void enqueue_set_velocity(bl_ctx* c, const float2* vraw);   // stationary state equation only
void op_set_velocity(bl_ctx* c, const float2* vraw);        // enqueue, synchronise, read E
void finish_set_velocity(bl_ctx* c);   // E from the published sums (after a sync)
// gradient into gout; with sq_part / max_part not NULL, also the finalize_blocks partials of
// |g|^2 and max |g| where the last kernel can form them (returns true then)
bool op_gradient(bl_ctx* c, float2* gout, double* sq_part = nullptr, double* max_part = nullptr);
// H draw into hout; with dot_part not NULL, also the finalize_blocks partials of <draw, hout>
// where the product's last kernel can form them (returns true then; false: not formed)
bool op_hessvec(bl_ctx* c, const float2* draw, float2* hout, double* dot_part = nullptr);
void vec_dot_partial(bl_ctx* c, const float2* a, const float2* b, double* pa);
void choose_launch_shapes(bl_ctx* c);
// the launch shapes chosen earlier in the process for this grid shape, else the defaults;
// no timing, no allocation
void apply_known_launch_shapes(bl_ctx* c);

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const DeviceError& e) {
    return fail(BL_E_DEVICE, std::string("HIP error in ") + e.where + ": " + hipGetErrorString(e.e));
  } catch (const NonFinite& e) {
    return fail(BL_E_NONFINITE, std::string("non-finite value in ") + e.what);
  } catch (const std::bad_alloc&) {
    return fail(BL_E_NOMEM, "device working set does not fit in free memory");
  } catch (...) {
    return fail(BL_E_DEVICE, "unexpected internal error");
  }
}

}  // namespace host
}  // namespace bl
