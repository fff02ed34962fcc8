// Gauss-Newton Hessian-vector product that allocates nothing: bl_lddmm_hessvec_noalloc.
//
// The same operation and kernels as bl_lddmm_hessvec (the product of Section 3.2 equation
// BLHessianStateEquation with the Gauss-Newton rule of Section 3.4), with the whole device
// working set of the call -- grid fields, offsets, stored states and adjoints, band vectors,
// transform buffers and twiddle tables, reduction partials and scalars -- placed in one
// file-scope device array instead of memory the library allocates.  Each device the library
// runs on holds its own copy of the array until the process ends; its device address is
// looked up once per device.  No published host scalars are used (the product needs none),
// no stream, event or pinned buffer is created, and launch shapes come from earlier tuning in
// the process or the defaults (tuning would create events).  Calls on one device share the
// array: they must not overlap (a second call while one runs on the same device races).
#include <mutex>

#include "bl_host.h"

namespace {

using namespace bl::host;

constexpr size_t kScratchBytes = size_t(512) << 20;   // 512 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up once per device, device current)
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

uint64_t bl_lddmm_noalloc_limit(void) { return (uint64_t)kScratchBytes; }

int bl_lddmm_hessvec_noalloc(const bl_problem* prob, const float* I0, const float* I1,
                             const float* v_hat, const float* dv_hat, float* hv_hat) {
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (!I0 || !I1 || !v_hat || !dv_hat || !hv_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  if (g.deform || g.nodes > 1)
    return fail(BL_E_UNSUPPORTED, "the allocation-free product serves the stationary "
                                  "state-equation model (no BL_NONSTATIONARY, BL_DEFORMATION)");
  const size_t need = ctx_bytes(g, true, false, prob->precision == BL_MIXED);
  if (need > kScratchBytes)
    return fail(BL_E_NOMEM, "problem needs " + std::to_string(need) + " bytes of scratch; the "
                            "allocation-free product is limited to " +
                            std::to_string(kScratchBytes) + " bytes");
  return guarded([&]() {
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device < 0 || device >= kMaxDevices) throw DeviceError{hipErrorInvalidDevice, "device index"};
    void* arena = scratch_address(device);
    const bool devptr = (prob->flags & BL_DEVICE_PTRS) != 0;
    hipStream_t s = devptr ? (hipStream_t)prob->stream : nullptr;
    CtxHolder h;
    h.c = create_ctx(prob, g, true, false, arena, kScratchBytes, s, nullptr, false);
    bl_ctx* c = h.c;
    apply_known_launch_shapes(c);
    load_images(c, I0, I1);
    load_band(c, v_hat, c->braw, g.dim);
    enqueue_set_velocity(c, c->braw);
    load_band(c, dv_hat, c->braw, g.dim);
    op_hessvec(c, c->braw, c->bout);
    store_band(c, c->bout, hv_hat, g.dim);
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (flag) throw NonFinite{"Hessian-vector product"};
    return BL_OK;
  });
}

}  // extern "C"
