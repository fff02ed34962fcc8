// C interface, device contexts and the Gauss-Newton-Krylov driver of the library.
//
// Host side of the hot path: argument validation (before any device call), the device
// arena of one registration problem, the operator sequences of the gradient (paper
// Section 3.2) and of the Gauss-Newton Hessian-vector product (Section 3.2 equation
// BLHessianStateEquation with the Gauss-Newton rule of Section 3.4), and the reduced-space
// solver (Section 3.4 equations BLNewton and BLKKT) with PCG preconditioned by K~ = L~^-1
// and Armijo backtracking.  All arithmetic runs in the kernels of the other translation
// units; this file only sequences launches, copies and scalar read-backs.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "bl_host.h"

namespace bl {
namespace host {

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

// ------------------------------------------------------------------------------ validation
int validate(const bl_problem* p, bl::Geo* g) {
  if (!p) return fail(BL_E_INVALID, "problem is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(BL_E_INVALID, "dim must be 2 or 3");
  int n[3] = {1, 1, 1}, k[3] = {1, 1, 1};
  for (int j = 0; j < p->dim; ++j) {
    n[j] = p->n[j];
    k[j] = p->k[j];
    if (n[j] < 4 || n[j] > 2048) return fail(BL_E_INVALID, "grid size n[j] must be in [4, 2048]");
    if (k[j] < 2 || (k[j] & 1) || k[j] > n[j])
      return fail(BL_E_INVALID, "band size k[j] must be even, >= 2 and <= n[j]");
  }
  if (p->dim == 3 && k[2] > 2 * bl::kMaxKzh)
    return fail(BL_E_INVALID, "band size k[2] must be <= 128");
  if ((int64_t)n[0] * n[1] * n[2] >= (int64_t(1) << 30))
    return fail(BL_E_INVALID, "grid must have fewer than 2^30 voxels");
  if (p->nt < 1 || p->nt > 256) return fail(BL_E_INVALID, "nt must be in [1, 256]");
  if (!std::isfinite(p->alpha) || p->alpha < 0) return fail(BL_E_INVALID, "alpha must be finite and >= 0");
  if (p->s < 0 || p->s > 8) return fail(BL_E_INVALID, "s must be in [0, 8]");
  if (!std::isfinite(p->sigma) || !(p->sigma > 0)) return fail(BL_E_INVALID, "sigma must be finite and > 0");
  if (p->gamma != 0 && p->gamma != 1) return fail(BL_E_INVALID, "gamma must be 0 or 1");
  if (p->precision != BL_FP32 && p->precision != BL_MIXED)
    return fail(BL_E_UNSUPPORTED, "precision must be BL_FP32 or BL_MIXED");
  if (p->flags & ~(BL_DEVICE_PTRS | BL_NEWTON | BL_NONSTATIONARY | BL_DEFORMATION))
    return fail(BL_E_INVALID, "unknown flag bits");
  if ((p->flags & BL_DEFORMATION) && (p->flags & (BL_NEWTON | BL_NONSTATIONARY)))
    return fail(BL_E_UNSUPPORTED,
                "the deformation state equation takes Gauss-Newton products of a stationary velocity only");
  if ((p->flags & BL_NEWTON) && (p->flags & BL_NONSTATIONARY))
    return fail(BL_E_UNSUPPORTED, "full Newton products of a non-stationary velocity are not supported");
  if (g) {
    g->dim = p->dim;
    g->nx = n[0]; g->ny = n[1]; g->nz = n[2];
    g->kx = k[0]; g->ky = k[1]; g->kz = k[2];
    g->kzh = p->dim == 3 ? k[2] / 2 : 1;
    g->kz0 = p->dim == 3 ? k[2] / 2 : 0;
    g->nt = p->nt;
    g->nref = std::max(n[0], std::max(n[1], n[2]));
    g->M = (int64_t)n[0] * n[1] * n[2];
    g->B = (int64_t)k[0] * k[1] * k[2];
    g->dt = (float)(1.0 / p->nt);
    g->half_nref = 0.5f * (float)g->nref;
    g->lam_scale = (float)(-2.0 / (p->sigma * p->sigma));
    g->inv_nx = 1.0f / (float)n[0];
    g->inv_ny = 1.0f / (float)n[1];
    g->inv_nz = 1.0f / (float)n[2];
    g->gamma = p->gamma;
    g->newton = (p->flags & BL_NEWTON) ? 1 : 0;
    g->nodes = (p->flags & BL_NONSTATIONARY) ? p->nt + 1 : 1;
    g->deform = (p->flags & BL_DEFORMATION) ? 1 : 0;
    // product grid of the truncated convolutions: 3 K / 2 points per axis rounded up to even
    // (at least 3 K / 2 - 2 keep every product term of two band fields from aliasing into the
    // band)
    auto pgrid = [](int kk) { const int v = 3 * kk / 2; return v + (v & 1); };
    g->px = pgrid(k[0]);
    g->py = pgrid(k[1]);
    g->pz = p->dim == 3 ? pgrid(k[2]) : 1;
    const bool d3 = p->dim == 3;
    g->zv[bl::TR_STATE] = d3 ? 2 : 1;
    g->zv[bl::TR_INC] = d3 ? 2 : 1;
    g->zv[bl::TR_ADJ] = d3 ? 2 : 1;
    g->zv[bl::TR_FORCE] = d3 ? 2 : 1;
    g->zv[bl::TR_SETUP] = 1;
    g->zv[bl::TR_IOTA_Z] = 1;
    g->zv[bl::TR_IOTA_XY] = 0;
    g->zv[bl::TR_CLASSES] = 0;
    g->stream_out = 9 * 4 * g->M > (int64_t(256) << 20) ? 1 : 0;
  }
  return BL_OK;
}

int validate_opts(const bl_solver_opts* o) {
  if (!o) return BL_OK;
  if (o->max_gn < 0 || o->max_gn > BL_MAX_GN) return fail(BL_E_INVALID, "max_gn must be in [0, 64]");
  if (o->max_pcg < 1 || o->max_pcg > 1000) return fail(BL_E_INVALID, "max_pcg must be in [1, 1000]");
  if (!std::isfinite(o->gtol) || o->gtol < 0) return fail(BL_E_INVALID, "gtol must be finite and >= 0");
  if (!std::isfinite(o->c1) || o->c1 < 0 || o->c1 >= 1) return fail(BL_E_INVALID, "c1 must be in [0, 1)");
  if (o->max_halvings < 0 || o->max_halvings > 60) return fail(BL_E_INVALID, "max_halvings must be in [0, 60]");
  return BL_OK;
}

// ------------------------------------------------------------------------------ arena
struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) & ~size_t(255);
    return off;
  }
};


}  // namespace host
}  // namespace bl


namespace bl {
namespace host {

size_t plane_bytes(const bl::Geo& g) { return (size_t)g.M * sizeof(float); }
size_t band_bytes(const bl::Geo& g) { return (size_t)g.B * sizeof(float2); }
// components of the widest transform: 4, or every node's velocity and divergence at once for a
// non-stationary velocity
size_t max_components(const bl::Geo& g) {
  return std::max<size_t>(4, g.nodes > 1 ? (size_t)g.nodes * (g.dim + 1) : 4);
}
size_t stage_elems(const bl::Geo& g) {
  return max_components(g) * g.kzh * (size_t)std::max<int64_t>((int64_t)g.ky * g.nx, (int64_t)g.ny * g.nx);
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }
int nyp_of(const bl::Geo& g) { return round_up(g.ny, 32); }
int kyp_of(const bl::Geo& g) { return round_up(g.ky, bl::kJG); }
int kxp_of(const bl::Geo& g) { return round_up(g.kx, 8); }
int nxp_of(const bl::Geo& g) { return round_up(g.nx, 8); }
int nzp_of(const bl::Geo& g) { return round_up(g.nz, 128); }

struct Offsets {
  size_t I1, m, X, YA, V, DV, T0, T1, L, Bf, DM, DL, U, braw, bv, bd, bout, P, Lhat, Lhat64, tw_x, tw_xT,
      tw_y, tw_yT, tw_zT, wi, wp, bufA, bufB, red, scal, flag, solver;
  // deformation state equation
  size_t IG, GP, UG, VP, DVP, DUG, GW, KG, GACC, DUb, US, ACC, KAP, RHO, ASUM, KSUM, PH, ptw_x,
      ptw_xT, ptw_y, ptw_yT, ptw_zT, pbufA, pbufB;
  size_t total;
};

// the product grid of the deformation method as a transform geometry (same band)
bl::Geo product_geo(const bl::Geo& g) {
  bl::Geo p = g;
  p.nx = g.px;
  p.ny = g.py;
  p.nz = g.pz;
  p.M = (int64_t)g.px * g.py * g.pz;
  p.nref = std::max(g.px, std::max(g.py, g.pz));
  p.inv_nx = 1.0f / (float)g.px;
  p.inv_ny = 1.0f / (float)g.py;
  p.inv_nz = 1.0f / (float)g.pz;
  p.half_nref = 0.5f * (float)p.nref;
  p.stream_out = 0;   // no transport runs on the product grid
  return p;
}

Offsets plan_layout(const bl::Geo& g, bool transport, bool solver, bool mixed) {
  Layout L;
  Offsets o{};
  const size_t pb = plane_bytes(g), bb = band_bytes(g);
  const int d = g.dim;
  const bool ns = g.nodes > 1;
  const size_t steps = ns ? (size_t)g.nt : 1;   // offset fields per time step (non-stationary)
  if (transport && g.deform) {
    const bl::Geo gp = product_geo(g);
    const size_t ppb = (size_t)gp.M * sizeof(float);
    const size_t d2 = (size_t)d * d;
    o.I1 = L.take(pb);
    o.m = L.take(pb * 2);          // I0, m(1)
    o.IG = L.take(pb * 4);
    o.GP = L.take(pb * 4);
    o.UG = L.take(pb * d);
    o.Bf = L.take(pb * d);
    o.VP = L.take(ppb * d);
    o.DVP = L.take(ppb * d);
    o.DUG = L.take(ppb * d2 * 4 * g.nt);
    o.GW = L.take(ppb * d2);
    o.KG = L.take(ppb * d);
    o.GACC = L.take(ppb * d);
    o.DUb = L.take(bb * d2);
    o.US = L.take(bb * 2 * d);
    o.ACC = L.take(bb * d);
    o.KAP = L.take(bb * d);
    o.RHO = L.take(bb * d);
    o.ASUM = L.take(bb * d);
    o.KSUM = L.take(bb * d);
    o.PH = L.take(d2 * g.kzh * g.ky * g.kx * sizeof(float2));
    o.ptw_x = L.take((size_t)kxp_of(gp) * gp.nx * sizeof(float2));
    o.ptw_xT = L.take((size_t)nxp_of(gp) * gp.kx * sizeof(float2));
    o.ptw_y = L.take((size_t)kyp_of(gp) * nyp_of(gp) * sizeof(float2));
    o.ptw_yT = L.take((size_t)nyp_of(gp) * kyp_of(gp) * sizeof(float2));
    o.ptw_zT = L.take((size_t)bl::kZP * nzp_of(gp) * sizeof(float2));
    // transform stage buffers for dim^2 components
    const size_t pst = std::max<size_t>(4, d2) * gp.kzh *
                       (size_t)std::max<int64_t>((int64_t)gp.ky * gp.nx, (int64_t)gp.ny * gp.nx);
    o.pbufA = L.take(pst * sizeof(float2));
    o.pbufB = L.take(pst * sizeof(float2));
  } else if (transport) {
    o.I1 = L.take(pb);
    o.m = L.take(pb * (g.nt + 1));
    o.X = L.take(pb * d * steps);
    o.YA = L.take(pb * 4 * steps);
    // non-stationary: every node's fields at once, so that each transform is one launch
    o.V = L.take(pb * (d + 1) * g.nodes);
    o.DV = L.take(pb * d * g.nodes);
    o.T0 = L.take(pb);
    o.T1 = L.take(pb);
    o.L = L.take(pb * (g.nt + 1));
    o.Bf = L.take(pb * d * g.nodes);
    if (g.newton) {   // dm^n, dlambda^n (Nt + 1 planes each) and the u ping-pong
      o.DM = L.take(pb * (g.nt + 1));
      o.DL = L.take(pb * (g.nt + 1));
      o.U = L.take(pb * 2);
    }
  } else {
    o.V = L.take(pb * 4);
  }
  const size_t vb = (size_t)g.nodes * d;   // band components of a velocity
  o.braw = L.take(bb * std::max<size_t>(4, vb));
  o.bv = L.take(bb * std::max<size_t>(4, (size_t)g.nodes * (d + 1)));
  o.bd = L.take(bb * std::max<size_t>(4, vb));
  o.bout = L.take(bb * std::max<size_t>(4, vb));
  o.P = L.take(max_components(g) * g.kzh * g.ky * g.kx * sizeof(float2));
  o.Lhat = L.take((size_t)g.B * sizeof(float));
  o.Lhat64 = L.take((size_t)g.B * sizeof(double));
  o.tw_x = L.take((size_t)kxp_of(g) * g.nx * sizeof(float2));
  o.tw_xT = L.take((size_t)nxp_of(g) * g.kx * sizeof(float2));
  o.tw_y = L.take((size_t)kyp_of(g) * nyp_of(g) * sizeof(float2));
  o.tw_yT = L.take((size_t)nyp_of(g) * kyp_of(g) * sizeof(float2));
  o.tw_zT = L.take((size_t)bl::kZP * nzp_of(g) * sizeof(float2));
  if (mixed) {
    o.wi = L.take((size_t)2 * round_up(g.nz, 32) * bl::mixed_kp(g) * sizeof(unsigned short));
    o.wp = L.take((size_t)2 * 32 * bl::mixed_jt(g) * round_up(g.nz, 16) * sizeof(unsigned short));
  }
  o.bufA = L.take(stage_elems(g) * sizeof(float2));
  o.bufB = L.take(stage_elems(g) * sizeof(float2));
  o.red = L.take((size_t)RED_SLOTS * bl::kRedBlocks * sizeof(double));
  o.scal = L.take(64 * sizeof(double));
  o.flag = L.take(256);
  o.solver = solver ? L.take(bb * vb * 8) : 0;
  o.total = L.total;
  return o;
}

// exp(+2 pi i k x / N) for centred (k = j - K/2) or plain (k = j) frequency indices, from the
// exactly reduced angle 2 pi ((k x) mod N) / N in FP64.
float2 twiddle(int j, int K, int x, int N, bool centred) {
  const double two_pi = 6.283185307179586476925286766559;
  const long long k = centred ? (long long)j - K / 2 : j;
  long long r = (k * x) % N;
  if (r < 0) r += N;
  const double ang = two_pi * (double)r / (double)N;
  return make_float2((float)std::cos(ang), (float)std::sin(ang));
}

// table[row][col] with `rows` x `cols` entries, zero outside j < K, x < N; transposed tables
// index [x][j].
void twiddles(std::vector<float2>& t, int rows, int cols, int K, int N, bool centred,
              bool transposed) {
  t.assign((size_t)rows * cols, make_float2(0.f, 0.f));
  for (int j = 0; j < K; ++j)
    for (int x = 0; x < N; ++x) {
      const size_t i = transposed ? (size_t)x * cols + j : (size_t)j * cols + x;
      t[i] = twiddle(j, K, x, N, centred);
    }
}

// FP32 value -> BF16 bits, round to nearest even
unsigned short bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
double bf16_value(unsigned short h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
// split hi/lo BF16 pair of an FP64 value
void split_bf16(double t, unsigned short& hi, unsigned short& lo) {
  hi = bf16_bits((float)t);
  lo = bf16_bits((float)(t - bf16_value(hi)));
}

// Matrices of the mixed-precision z stages (exactly reduced angles in FP64, split to BF16):
//   Wi[z][2h] = s_h cos(2 pi h z / nz), Wi[z][2h+1] = -s_h sin(..), s_0 = 1, s_h = 2, rows
//   z < round_up(nz, 32), columns < mixed_kp;  Wp[2h][z] = cos(..), Wp[2h+1][z] = -sin(..),
//   rows < 32 mixed_jt, columns z < round_up(nz, 16).  Each as a hi table followed by a lo
//   table; entries outside h < kzh, z < nz are zero.
void mixed_tables(const bl::Geo& g, std::vector<unsigned short>& wi,
                  std::vector<unsigned short>& wp) {
  const double two_pi = 6.283185307179586476925286766559;
  const int kp = bl::mixed_kp(g), zi = round_up(g.nz, 32);
  const int jr = 32 * bl::mixed_jt(g), zp = round_up(g.nz, 16);
  wi.assign((size_t)2 * zi * kp, 0);
  wp.assign((size_t)2 * jr * zp, 0);
  for (int z = 0; z < g.nz; ++z)
    for (int h = 0; h < g.kzh; ++h) {
      long long r = ((long long)h * z) % g.nz;
      const double ang = two_pi * (double)r / (double)g.nz;
      const double cs = std::cos(ang), sn = std::sin(ang), sh = h == 0 ? 1.0 : 2.0;
      unsigned short hi, lo;
      split_bf16(sh * cs, hi, lo);
      wi[(size_t)z * kp + 2 * h] = hi;
      wi[(size_t)zi * kp + (size_t)z * kp + 2 * h] = lo;
      split_bf16(-sh * sn, hi, lo);
      wi[(size_t)z * kp + 2 * h + 1] = hi;
      wi[(size_t)zi * kp + (size_t)z * kp + 2 * h + 1] = lo;
      split_bf16(cs, hi, lo);
      wp[(size_t)(2 * h) * zp + z] = hi;
      wp[(size_t)jr * zp + (size_t)(2 * h) * zp + z] = lo;
      split_bf16(-sn, hi, lo);
      wp[(size_t)(2 * h + 1) * zp + z] = hi;
      wp[(size_t)jr * zp + (size_t)(2 * h + 1) * zp + z] = lo;
    }
}

double* alloc_host_scalars() {
  // coherent: kernels store straight to host memory, visible once the stream has synchronised
  double* h = nullptr;
  HIP_TRY(hipHostMalloc((void**)&h, 64 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  for (int i = 0; i < 64; ++i) h[i] = 0.0;
  return h;
}

void destroy_ctx(bl_ctx* c) {
  if (!c) return;
  // best-effort teardown: errors here have nowhere to go
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->arena && c->own_arena) (void)hipFree(c->arena);
  if (c->hscal && c->own_hscal) (void)hipHostFree(c->hscal);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

bl_ctx* create_ctx(const bl_problem* prob, const bl::Geo& g, bool transport, bool solver,
                   void* arena, size_t arena_bytes, hipStream_t stream, double* host_scalars,
                   bool host_mirror) {
  bl_ctx* c = new bl_ctx();
  try {
    c->g = g;
    c->prob = *prob;
    c->devptr = (prob->flags & BL_DEVICE_PTRS) != 0;
    c->transport = transport;
    HIP_TRY(hipGetDevice(&c->device));
    if (arena) {
      c->stream = stream;          // caller-owned arena and stream
      c->own_stream = false;
    } else if (c->devptr) {
      c->stream = (hipStream_t)prob->stream;
      c->own_stream = false;
    } else {
      HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    const bool mixed = prob->precision == BL_MIXED;
    const Offsets o = plan_layout(g, transport, solver, mixed);
    if (arena) {
      if (arena_bytes < o.total) throw std::bad_alloc();
      c->arena = static_cast<char*>(arena);
      c->own_arena = false;
    } else {
      size_t free_b = 0, total_b = 0;
      HIP_TRY(hipMemGetInfo(&free_b, &total_b));
      if (o.total + (64u << 20) > free_b) throw std::bad_alloc();
      HIP_TRY(hipMalloc(&c->arena, o.total));
      c->own_arena = true;
    }
    c->arena_bytes = o.total;
    char* a = c->arena;
    auto F = [&](size_t off) { return reinterpret_cast<float*>(a + off); };
    auto C2 = [&](size_t off) { return reinterpret_cast<float2*>(a + off); };
    auto F4 = [&](size_t off) { return reinterpret_cast<float4*>(a + off); };
    if (transport && g.deform) {
      c->I1 = F(o.I1); c->m = F(o.m); c->mfinal = c->m + g.M;
      c->IG = F4(o.IG); c->GP = F4(o.GP); c->UG = F(o.UG); c->Bf = F(o.Bf);
      c->gP = product_geo(g);
      c->VP = F(o.VP); c->DVP = F(o.DVP); c->DUG = F(o.DUG); c->GW = F(o.GW); c->KG = F(o.KG);
      c->GACC = F(o.GACC);
      c->DUb = C2(o.DUb); c->US = C2(o.US); c->ACC = C2(o.ACC); c->KAP = C2(o.KAP);
      c->RHO = C2(o.RHO); c->ASUM = C2(o.ASUM); c->KSUM = C2(o.KSUM); c->PH = C2(o.PH);
      bl::DftPlan& q = c->planP;
      q.tw_x = C2(o.ptw_x); q.tw_xT = C2(o.ptw_xT); q.tw_y = C2(o.ptw_y); q.tw_yT = C2(o.ptw_yT);
      q.tw_zT = C2(o.ptw_zT);
      q.nyp = nyp_of(c->gP); q.kyp = kyp_of(c->gP); q.kxp = kxp_of(c->gP);
      q.nxp = nxp_of(c->gP); q.nzp = nzp_of(c->gP);
      q.bufA = C2(o.pbufA); q.bufB = C2(o.pbufB);
      q.mixed = 0;
      const char* fenv = std::getenv("BL_DEFORM_FUSED");
      c->fused = bl::fused_ok(g, c->gP) && !(fenv && fenv[0] == '0');
    } else if (transport) {
      c->I1 = F(o.I1); c->m = F(o.m); c->mfinal = c->m + (size_t)g.nt * g.M;
      c->X = F(o.X);
      c->YA = reinterpret_cast<float4*>(a + o.YA);
      c->DV = F(o.DV);
      c->T0 = F(o.T0); c->T1 = F(o.T1); c->L = F(o.L); c->Bf = F(o.Bf);
      if (g.newton) {
        c->DM = F(o.DM); c->DL = F(o.DL); c->U0 = F(o.U); c->U1 = F(o.U) + g.M;
      }
    }
    if (!g.deform || !transport) c->V = F(o.V);
    c->braw = C2(o.braw); c->bv = C2(o.bv); c->bd = C2(o.bd); c->bout = C2(o.bout); c->P = C2(o.P);
    c->Lhat = F(o.Lhat);
    c->Lhat64 = reinterpret_cast<double*>(a + o.Lhat64);
    c->plan.tw_x = C2(o.tw_x); c->plan.tw_xT = C2(o.tw_xT);
    c->plan.tw_y = C2(o.tw_y); c->plan.tw_yT = C2(o.tw_yT); c->plan.tw_zT = C2(o.tw_zT);
    c->plan.nyp = nyp_of(g); c->plan.kyp = kyp_of(g); c->plan.kxp = kxp_of(g);
    c->plan.nxp = nxp_of(g); c->plan.nzp = nzp_of(g);
    c->plan.bufA = C2(o.bufA); c->plan.bufB = C2(o.bufB);
    c->plan.mixed = mixed;
    if (mixed) {
      c->plan.wi_bf16 = reinterpret_cast<unsigned short*>(a + o.wi);
      c->plan.wp_bf16 = reinterpret_cast<unsigned short*>(a + o.wp);
      c->plan.nzp32 = round_up(g.nz, 32);
      c->plan.nzp16 = round_up(g.nz, 16);
    }
    c->red = reinterpret_cast<double*>(a + o.red);
    c->scal = reinterpret_cast<double*>(a + o.scal);
    c->flag = reinterpret_cast<int*>(a + o.flag);
    if (solver) {
      float2* s = C2(o.solver);
      const size_t nb = (size_t)g.nodes * g.dim * g.B;
      c->sv = s; c->sg = s + nb; c->sdelta = s + 2 * nb; c->sr = s + 3 * nb; c->sz = s + 4 * nb;
      c->sp = s + 5 * nb; c->sHp = s + 6 * nb; c->stry = s + 7 * nb;
    }
    if (!host_mirror) {
      c->hscal = nullptr;
      c->hdev = nullptr;
      c->own_hscal = false;
    } else if (host_scalars) {
      c->hscal = host_scalars;
      c->own_hscal = false;
    } else {
      c->hscal = alloc_host_scalars();
    }
    if (c->hscal) HIP_TRY(hipHostGetDevicePointer((void**)&c->hdev, c->hscal, 0));
    // host tables: twiddles of exactly reduced angles, the symbol of L
    std::vector<float2> tw;
    auto upload = [&](float2* dst) {
      HIP_TRY(hipMemcpyAsync(dst, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    };
    auto tables = [&](const bl::Geo& gg, bl::DftPlan& pl) {
      twiddles(tw, pl.kxp, gg.nx, gg.kx, gg.nx, true, false);
      upload(pl.tw_x);
      twiddles(tw, pl.nxp, gg.kx, gg.kx, gg.nx, true, true);
      upload(pl.tw_xT);
      twiddles(tw, pl.kyp, pl.nyp, gg.ky, gg.ny, true, false);
      upload(pl.tw_y);
      twiddles(tw, pl.nyp, pl.kyp, gg.ky, gg.ny, true, true);
      upload(pl.tw_yT);
      twiddles(tw, pl.nzp, bl::kZP, gg.kzh, gg.nz, false, true);
      upload(pl.tw_zT);
    };
    tables(g, c->plan);
    if (c->DUG) tables(c->gP, c->planP);
    if (mixed) {
      std::vector<unsigned short> wi, wp;
      mixed_tables(g, wi, wp);
      HIP_TRY(hipMemcpyAsync(c->plan.wi_bf16, wi.data(), wi.size() * 2, hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(c->plan.wp_bf16, wp.data(), wp.size() * 2, hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    }
    std::vector<double> L64((size_t)g.B);
    std::vector<float> L32((size_t)g.B);
    const double four_pi2 = 39.478417604357434;
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (int64_t b = 0; b < g.B; ++b) {
      const int jx = (int)(b % g.kx), jy = (int)((b / g.kx) % g.ky), jz = (int)(b / ((int64_t)g.kx * g.ky));
      const int kv[3] = {jx - g.kx / 2, jy - g.ky / 2, jz - g.kz0};
      double q2 = 0;
      for (int j = 0; j < g.dim; ++j) {
        const double q = (double)kv[j] * (double)g.nref / (double)nn[j];
        q2 += q * q;
      }
      const double base = 1.0 + four_pi2 * prob->alpha * q2;
      double L = 1.0;
      for (int i = 0; i < prob->s; ++i) L *= base;
      L64[b] = L;
      L32[b] = (float)L;
    }
    HIP_TRY(hipMemcpyAsync(c->Lhat64, L64.data(), L64.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->Lhat, L32.data(), L32.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->flag, 0, 256, c->stream));
    if (c->DM) HIP_TRY(hipMemsetAsync(c->DM, 0, plane_bytes(g), c->stream));   // dm^0 = 0
    HIP_TRY(hipStreamSynchronize(c->stream));
  } catch (...) {
    destroy_ctx(c);
    throw;
  }
  return c;
}

inline hipMemcpyKind in_kind(const bl_ctx* c) {
  return c->devptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
void sync(bl_ctx* c) { HIP_TRY(hipStreamSynchronize(c->stream)); }

// -------------------------------------------------------------------------------- timing
// Timed launches record a HIP event pair at their kernel's own start and end (the dispatch
// timestamps): the durations are those of the kernels alone, as a kernel trace reports them.
}  // namespace host
thread_local LaunchEvents* t_next_launch = nullptr;
void set_launch_events(LaunchEvents* e) { t_next_launch = e; }
LaunchEvents* take_launch_events() {
  LaunchEvents* e = t_next_launch;
  t_next_launch = nullptr;
  return e;
}
namespace host {

// arm the next BL_LAUNCH on this thread with an event pair of the pool, counted for class cls;
// false when the pool is used up (the launch is then not timed)
bool t_arm(bl_ctx* c, int cls) {
  if (!c->timing || c->ev_next + 2 > c->ev_pool.size()) return false;
  bl::LaunchEvents& e = c->ev_pairs[c->ev_next / 2];
  e.start = c->ev_pool[c->ev_next];
  e.stop = c->ev_pool[c->ev_next + 1];
  bl::set_launch_events(&e);
  c->ev_used.push_back({cls, (int)c->ev_next, 1});
  c->ev_next += 2;
  return true;
}

// f() with its first BL_LAUNCH timed for class cls while timing is on.  A pair that f did not
// use (it threw first, or launched nothing through BL_LAUNCH) is disarmed and forgotten, so it
// can neither time an unrelated later launch nor be read unrecorded.
template <class F>
void timed(bl_ctx* c, int cls, F&& f) {
  if (!c->timing) {
    f();
    return;
  }
  struct Disarm {
    bl_ctx* c;
    bool armed;
    ~Disarm() {
      if (bl::take_launch_events() != nullptr && armed) {
        c->ev_used.pop_back();
        c->ev_next -= 2;
      }
    }
  } d{c, t_arm(c, cls)};
  f();
}
void t_collect(bl_ctx* c) {
  if (c->ev_used.empty()) return;
  sync(c);
  for (const auto& u : c->ev_used) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[u.ev], c->ev_pool[u.ev + 1]));
    c->t_launch[u.cls] += u.count;
    c->t_ms[u.cls] += ms;
  }
  c->ev_used.clear();
  c->ev_next = 0;
}

// ------------------------------------------------------------------------------ operators
// ------------------------------------------------------------------ transport launch shapes
// Launch shapes, chosen per problem shape by timing and remembered (the autotuner).
//
// Every class's candidates compute bitwise the same values -- they only change how work is
// split over threads and blocks -- so tuning never changes a result:
//   transports (state, incremental, adjoint, body force) and setup: voxels per thread along z
//     (tiles of 64 x 4 x zv voxels), 1, 2, 4 or 8;
//   iota z stage (FP32): the z-chunk multiplier of its grid, 1, 2 or 4;
//   iota x and y stages: two kernels (0) or one fused kernel with 32 or 16 rows per block.
// Candidates are timed on the context's own fields right after the first setup on a problem
// shape (the gathers' cache behaviour depends on the real offsets); the planes they write
// (T0, T1, Bf, DV, X, YA with the same values, the transform buffers) are work space that every
// operation rewrites before use.  Choices are kept per (GPU architecture, grid, band,
// precision) for the process and in a cache file -- BL_TUNE_CACHE, else
// $XDG_CACHE_HOME/bl_lddmm/launch_shapes_v2.txt or ~/.cache/bl_lddmm/launch_shapes_v2.txt -- read at
// the first tuning and appended to after each new choice, so later processes skip the timing.
// BL_TUNE_CACHE=off disables the file; BL_TRANSPORT_ZV = 1, 2, 4 or 8 fixes the transports'
// and the setup's voxels per thread and skips the timing, BL_LAUNCH_SHAPES fixes every class.
std::mutex g_shape_mu;
std::map<std::string, std::array<int, bl::TR_CLASSES>> g_shapes;
bool g_shapes_file_read = false;

std::string tune_cache_path() {
  const char* e = std::getenv("BL_TUNE_CACHE");
  if (e && *e) return std::string(e) == "off" ? std::string() : std::string(e);
  if (const char* x = std::getenv("XDG_CACHE_HOME"))
    if (*x) return std::string(x) + "/bl_lddmm/launch_shapes_v2.txt";
  if (const char* h = std::getenv("HOME"))
    if (*h) return std::string(h) + "/.cache/bl_lddmm/launch_shapes_v2.txt";
  return std::string();
}

std::string shape_key(const bl_ctx* c) {
  static std::string arch = []() {
    hipDeviceProp_t pr{};
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || hipGetDeviceProperties(&pr, d) != hipSuccess)
      return std::string("unknown");
    std::string a = pr.gcnArchName;
    return a.substr(0, a.find(':'));
  }();
  const bl::Geo& g = c->g;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s %d %d %d %d %d %d %d %d", arch.c_str(), g.dim, g.nx, g.ny,
                g.nz, g.kx, g.ky, g.kz, c->plan.mixed);
  return buf;
}

// a launch-shape list every class accepts: voxels per thread 1, 2, 4 or 8 for the transports
// and the setup, 1, 2 or 4 for the iota z chunking, 0, 16 or 32 for the iota x/y stages
bool valid_shapes(const int* v) {
  bool ok = true;
  for (int k = 0; ok && k <= bl::TR_SETUP; ++k) ok = v[k] == 1 || v[k] == 2 || v[k] == 4 || v[k] == 8;
  ok = ok && (v[bl::TR_IOTA_Z] == 1 || v[bl::TR_IOTA_Z] == 2 || v[bl::TR_IOTA_Z] == 4);
  return ok && (v[bl::TR_IOTA_XY] == 0 || v[bl::TR_IOTA_XY] == 16 || v[bl::TR_IOTA_XY] == 32);
}

// the cache file's lines: "<arch> dim nx ny nz kx ky kz mixed : s0 ... s6"; malformed lines and
// lines with a value outside valid_shapes are skipped (caller holds g_shape_mu)
void read_shape_file() {
  g_shapes_file_read = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char* colon = std::strchr(line, ':');
    if (!colon) continue;
    std::string key(line, colon - line);
    while (!key.empty() && key.back() == ' ') key.pop_back();
    std::array<int, bl::TR_CLASSES> v{};
    int n = 0, off = 0;
    const char* q = colon + 1;
    while (n < bl::TR_CLASSES && std::sscanf(q, "%d%n", &v[n], &off) == 1) {
      q += off;
      ++n;
    }
    if (n == bl::TR_CLASSES && valid_shapes(v.data())) g_shapes[key] = v;
  }
  std::fclose(f);
}

void append_shape_file(const std::string& key, const std::array<int, bl::TR_CLASSES>& v) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos) {   // create the directory chain (errors ignored)
    for (size_t i = 1; i <= slash; ++i)
      if (path[i] == '/' || i == slash) ::mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
  }
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s :", key.c_str());
  for (int k = 0; k < bl::TR_CLASSES; ++k) std::fprintf(f, " %d", v[k]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

bool lookup_shapes(bl_ctx* c) {
  const std::string key = shape_key(c);
  std::lock_guard<std::mutex> lk(g_shape_mu);
  if (!g_shapes_file_read) read_shape_file();
  auto it = g_shapes.find(key);
  if (it == g_shapes.end()) return false;
  for (int k = 0; k < bl::TR_CLASSES; ++k) c->g.zv[k] = it->second[k];
  return true;
}

void apply_known_launch_shapes(bl_ctx* c) {
  c->tuned = true;
  if (c->g.dim != 3 || !c->transport) return;
  lookup_shapes(c);
}

bool body_forms_lambda0(const bl::Geo& g);

void choose_launch_shapes(bl_ctx* c) {
  c->tuned = true;
  bl::Geo& g = c->g;
  if (g.dim != 3 || !c->transport) return;
  // BL_LAUNCH_SHAPES = "s0,...,s6" fixes every class (tests of the shapes' equivalence);
  // an invalid list keeps the defaults
  if (const char* all = std::getenv("BL_LAUNCH_SHAPES")) {
    int v[bl::TR_CLASSES], n = 0, off = 0;
    const char* q = all;
    while (n < bl::TR_CLASSES && std::sscanf(q, "%d%n", &v[n], &off) == 1) {
      q += off;
      if (*q == ',') ++q;
      ++n;
    }
    if (n == bl::TR_CLASSES && valid_shapes(v))
      for (int k = 0; k < bl::TR_CLASSES; ++k) g.zv[k] = v[k];
    return;
  }
  const char* env = std::getenv("BL_TRANSPORT_ZV");
  if (env && *env) {
    const int v = std::atoi(env);
    if (v == 1 || v == 2 || v == 4 || v == 8)
      for (int k = 0; k <= bl::TR_SETUP; ++k) g.zv[k] = v;
    return;  // any other value keeps the defaults
  }
  if (lookup_shapes(c)) return;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  auto launch = [&](int cls) {
    switch (cls) {
      case bl::TR_STATE: bl::state_step(g, c->m, c->X, c->T0, s); break;
      case bl::TR_INC: bl::inc_step(g, c->T0, c->X, c->m + M, c->DV, c->T1, s); break;
      case bl::TR_ADJ: bl::adj_step(g, c->T0, c->YA, c->T1, s); break;
      case bl::TR_FORCE:
        bl::body_force(g, c->L, c->m, c->Bf, s, body_forms_lambda0(g) ? c->YA : nullptr);
        break;
      case bl::TR_SETUP: bl::setup(g, c->V, c->X, c->YA, s); break;   // same values again
      case bl::TR_IOTA_Z: bl::iota_z(g, c->plan, g.dim, c->DV, s); break;
      default: bl::iota_xy(g, c->plan, c->bv, g.dim, s); break;
    }
  };
  auto candidates = [&](int cls) -> std::vector<int> {
    switch (cls) {
      // (a non-stationary velocity has per-step offsets from its own setup kernel: the
      // stationary setup is not timed on its fields)
      case bl::TR_SETUP: return g.nodes > 1 ? std::vector<int>{} : std::vector<int>{1, 2, 4};
      case bl::TR_IOTA_Z: return c->plan.mixed ? std::vector<int>{} : std::vector<int>{1, 2, 4};
      // the fused iota x/y kernel times faster alone than the two stages (15.0 against
      // 17.4 us per launch at 128^3) but runs slower inside products and registrations (25 us
      // per call in a kernel trace, 2% fewer products per second), so timing it alone would
      // choose wrongly: not a candidate (BL_LAUNCH_SHAPES still selects it)
      case bl::TR_IOTA_XY: return {};
      default: return {1, 2, 4, 8};
    }
  };
  // Every candidate is launched once first; then the candidates are timed in turn, kRounds
  // times over, and each keeps its fastest round.  Interleaving keeps a clock ramp or a
  // neighbour's load from favouring whichever candidate is timed last.
  constexpr int kReps = 4, kRounds = 3;
  // BL_TUNE_LOG=1 prints every class's candidate times (per launch) and the choice to stderr
  const char* log_env = std::getenv("BL_TUNE_LOG");
  const bool log = log_env && *log_env && std::strcmp(log_env, "0") != 0;
  std::array<int, bl::TR_CLASSES> best;
  for (int cls = 0; cls < bl::TR_CLASSES; ++cls) {
    const int dflt = g.zv[cls];
    best[cls] = dflt;
    const std::vector<int> cand = candidates(cls);
    if (cand.empty()) continue;
    std::vector<int> order{dflt};
    for (int v : cand)
      if (v != dflt) order.push_back(v);
    for (int zv : order) {
      g.zv[cls] = zv;
      launch(cls);  // warm-up
    }
    std::vector<float> t_min(order.size(), std::numeric_limits<float>::infinity());
    for (int round = 0; round < kRounds; ++round)
      for (size_t i = 0; i < order.size(); ++i) {
        g.zv[cls] = order[i];
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < kReps; ++r) launch(cls);
        HIP_TRY(hipEventRecord(e1, s));
        check_launch("launch shape timing");
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        t_min[i] = std::min(t_min[i], ms);
      }
    // another shape must beat the default by 5% to replace it: timing noise, and a launch
    // timed alone runs on caches its neighbours in a product would have evicted (the body
    // force at 128^3 times 3.4% faster alone at one voxel per thread than at two, and runs
    // 2.5% slower inside products)
    float t_best = t_min[0];
    for (size_t i = 1; i < order.size(); ++i)
      if (t_min[i] < 0.95f * t_best) {
        t_best = t_min[i];
        best[cls] = order[i];
      }
    g.zv[cls] = best[cls];
    if (log) {
      std::fprintf(stderr, "[bl_lddmm tune] class %d:", cls);
      for (size_t i = 0; i < order.size(); ++i)
        std::fprintf(stderr, " %d=%.2fus", order[i], 1e3f * t_min[i] / kReps);
      std::fprintf(stderr, " -> %d\n", best[cls]);
    }
  }
  const std::string key = shape_key(c);
  std::lock_guard<std::mutex> lk(g_shape_mu);
  if (g_shapes.emplace(key, best).second) append_shape_file(key, best);
}

// ------------------------------------------------ non-stationary velocity (one field per node)
// Per node: projection (and divergence) of the band fields with the trapezoid-weighted
// regulariser; iota of every node's velocity and divergence in one launch sequence; per step
// t_n -> t_{n+1}: the step's offsets from both ends, and the state step.
void op_set_velocity_ns(bl_ctx* c, const float2* vraw) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M, B = (size_t)g.B;
  const int d = g.dim;
  double* red_reg = c->red + RED_REG * bl::kRedBlocks;
  double* red_data = c->red + RED_DATA * bl::kRedBlocks;
  for (int n = 0; n <= g.nt; ++n) {
    const double w = (n == 0 || n == g.nt) ? 0.5 / g.nt : 1.0 / g.nt;
    bl::band_prep(g, vraw + (size_t)n * d * B, c->bv + (size_t)n * (d + 1) * B, 1, c->Lhat64,
                  red_reg, s, w, n > 0);
  }
  // (v^n, r^n) of every node in one transform: V[n][c]
  bl::iota(g, c->plan, c->bv, (g.nt + 1) * (d + 1), c->V, s);
  // every step's offsets in one launch, then the state steps
  bl::setup_ns(g, c->V, c->X, c->YA, g.nt, s);
  if (!c->tuned) choose_launch_shapes(c);
  for (int n = 0; n < g.nt; ++n)
    bl::state_step(g, c->m + n * M, c->X + (size_t)n * d * M, c->m + (n + 1) * M, s);
  bl::energy_partial(g, c->m + g.nt * M, c->I1, red_data, s);
  bl::reduce_final2(red_reg, c->scal + S_REG, c->hdev + S_REG, red_data, c->scal + S_DATA,
                    c->hdev + S_DATA, bl::kRedBlocks, s);
  check_launch("set_velocity (non-stationary)");
  sync(c);
  c->reg = c->hscal[S_REG];
  c->data_sum = c->hscal[S_DATA];
  const double sig = c->prob.sigma;
  c->E = 0.5 * c->reg + c->data_sum / (sig * sig * (double)g.M);
  c->have_v = true;
  c->have_lambda = false;
  if (!std::isfinite(c->E)) throw NonFinite{"energy"};
}

// adjoint from L[nt] down to L[1] with the per-step (Y, a): lambda^0 is read by nothing but
// the per-node body force, whose node-0 blocks form it from lambda^1 (per_node_outputs) in
// parallel with the other nodes' blocks -- one launch and the plane's store and reload fewer
void backward_ns(bl_ctx* c) {
  const bl::Geo& g = c->g;
  const size_t M = (size_t)g.M;
  for (int n = g.nt - 1; n >= 1; --n)
    bl::adj_step(g, c->L + (n + 1) * M, c->YA + (size_t)n * M, c->L + n * M, c->stream);
}

// per node: b^n = L[n] grad m^n (every node's planes, then one pi), and the band output
// L^ vproj^n + pi(b^n)
void per_node_outputs(bl_ctx* c, const float2* vproj, size_t vstride, float2* out) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t B = (size_t)g.B;
  const int d = g.dim;
  bl::body_nodes(g, c->L, c->m, c->Bf, g.nt + 1, s, c->YA);   // YA of step 0: lambda^0
  bl::pi_half(g, c->plan, c->Bf, (g.nt + 1) * d, c->P, s);
  const size_t ph = (size_t)g.kzh * g.ky * g.kx;
  bl::band_finalize_nodes(g, d, vproj, vstride, c->Lhat, c->P, (size_t)d * ph,
                          (float)(1.0 / (double)g.M), out, (size_t)d * B, g.nt + 1, c->flag, s, 1);
}

void op_gradient_ns(bl_ctx* c, float2* gout) {
  const bl::Geo& g = c->g;
  const size_t M = (size_t)g.M;
  bl::terminal(g, c->m + g.nt * M, c->I1, c->L + g.nt * M, c->stream);
  backward_ns(c);
  c->have_lambda = true;
  per_node_outputs(c, c->bv, (size_t)(g.dim + 1) * g.B, gout);
  check_launch("gradient (non-stationary)");
}

void op_hessvec_ns(bl_ctx* c, const float2* draw, float2* hout) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M, B = (size_t)g.B;
  const int d = g.dim;
  bl::band_prep_nodes(g, draw, c->bd, g.nt + 1, (size_t)d * B, s);
  // every node's dv^n in one transform: DV[n][c]
  bl::iota(g, c->plan, c->bd, (g.nt + 1) * d, c->DV, s);
  bl::inc_init(g, c->m, c->DV, c->T0, s);
  float* tin = c->T0;
  float* tout = c->T1;
  for (int n = 0; n + 1 < g.nt; ++n) {
    bl::inc_step(g, tin, c->X + (size_t)n * d * M, c->m + (n + 1) * M,
                 c->DV + (size_t)(n + 1) * d * M, tout, s);
    std::swap(tin, tout);
  }
  bl::inc_last(g, tin, c->X + (size_t)(g.nt - 1) * d * M, c->m + g.nt * M,
               c->DV + (size_t)g.nt * d * M, c->L + g.nt * M, s);
  backward_ns(c);
  c->have_lambda = false;   // L holds the incremental adjoint now
  c->lamT_valid = false;
  per_node_outputs(c, c->bd, (size_t)d * B, hout);
  check_launch("hessvec (non-stationary)");
}

// ------------------------------------------------ deformation state equation (Section 3.3)
// Every stage of the band Runge-Kutta sweep: iota of the stage state's spectral derivatives
// onto the product grid, the pointwise products with iota(v~) (and, in products, of the stored
// stage derivatives with iota(dv~)), pi back to the band, and the band stage update.
float2* us_slot(bl_ctx* c, int k) { return c->US + (size_t)k * c->g.dim * c->g.B; }
float* dug_slot(bl_ctx* c, int n, int st) {
  const size_t d2 = (size_t)c->g.dim * c->g.dim;
  return c->DUG + (size_t)(n * 4 + (st - 1)) * d2 * (size_t)c->gP.M;
}

// from u~(0) = 0 (state) or du~(0) = 0 (incremental, source dv~ in bd); returns u~(1) / du~(1)
const float2* def_sweep_forward(bl_ctx* c, bool incremental) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const int d = g.dim, d2 = d * d;
  const int64_t MP = c->gP.M;
  const float scaleP = (float)(1.0 / (double)MP);
  const float2* src = incremental ? c->bd : c->bv;
  HIP_TRY(hipMemsetAsync(us_slot(c, 0), 0, band_bytes(g) * d, s));
  if (c->fused) {
    // three launches per stage; the stage state U_st is u_n (st = 1) or the state written by
    // the previous stage into DUb (used as a dim-field buffer here)
    const bl::DftPlan& pl = c->planP;
    int cur = 0;
    for (int n = 0; n < g.nt; ++n)
      for (int st = 1; st <= 4; ++st) {
        const float2* state = st == 1 ? us_slot(c, cur) : c->DUb;
        bl::fx_iota_xy(g, c->gP, pl, state, 1, pl.bufA, s);
        bl::fx_col_fwd(c->gP, pl, pl.bufA, c->VP, incremental ? nullptr : dug_slot(c, n, st),
                       incremental ? dug_slot(c, n, st) : nullptr, incremental ? c->DVP : nullptr,
                       pl.bufB, s);
        bl::fx_pi_yx_stage(g, c->gP, pl, pl.bufB, scaleP, src, us_slot(c, cur), c->ACC, st,
                           st == 4 ? us_slot(c, cur ^ 1) : c->DUb, s);
        if (st == 4) cur ^= 1;
      }
    return us_slot(c, cur);
  }
  HIP_TRY(hipMemsetAsync(c->DUb, 0, band_bytes(g) * d2, s));
  int cur = 0;
  for (int n = 0; n < g.nt; ++n)
    for (int st = 1; st <= 4; ++st) {
      float* dg = incremental ? c->GW : dug_slot(c, n, st);
      bl::iota(c->gP, c->planP, c->DUb, d2, dg, s);
      if (incremental) bl::def_prod(g, MP, dg, c->VP, dug_slot(c, n, st), c->DVP, c->KG, s);
      else bl::def_prod(g, MP, dg, c->VP, nullptr, nullptr, c->KG, s);
      bl::pi_half(c->gP, c->planP, c->KG, d, c->PH, s);
      const bool last = n + 1 == g.nt && st == 4;
      bl::def_stage(g, scaleP, c->PH, src, us_slot(c, cur), c->ACC, st, us_slot(c, cur ^ 1),
                    last ? nullptr : c->DUb, s);
      if (st == 4) cur ^= 1;
    }
  return us_slot(c, cur);
}

// the transposed sweep from rho~(1) in RHO; out = Lhat vproj + int (I + D~U)^T * rho~ dt
void def_sweep_backward(bl_ctx* c, const float2* vproj, float2* out) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const int d = g.dim, d2 = d * d;
  const int64_t MP = c->gP.M;
  const float scaleP = (float)(1.0 / (double)MP);
  bl::def_adj_init(g, c->RHO, c->KAP, c->KSUM, s);
  if (c->fused) {
    const bl::DftPlan& pl = c->planP;
    for (int n = g.nt - 1; n >= 0; --n)
      for (int st = 4; st >= 1; --st) {
        bl::fx_iota_xy(g, c->gP, pl, c->KAP, 0, pl.bufA, s);
        bl::fx_col_bwd(c->gP, pl, pl.bufA, c->VP, dug_slot(c, n, st), c->GACC,
                       n + 1 == g.nt && st == 4, pl.bufB, s);
        bl::fx_pi_yx_adj(g, c->gP, pl, pl.bufB, scaleP, c->RHO, c->ASUM, c->KSUM, c->KAP, st,
                         n > 0, s);
      }
    bl::pi_half(c->gP, c->planP, c->GACC, d, c->PH, s);
    bl::def_out(g, scaleP, c->PH, c->KSUM, vproj, c->Lhat, out, c->flag, s);
    return;
  }
  for (int n = g.nt - 1; n >= 0; --n)
    for (int st = 4; st >= 1; --st) {
      bl::iota(c->gP, c->planP, c->KAP, d, c->KG, s);
      bl::def_adj_prod(g, MP, c->KG, c->VP, dug_slot(c, n, st), c->GW, c->GACC,
                       n + 1 == g.nt && st == 4, s);
      bl::pi_half(c->gP, c->planP, c->GW, d2, c->PH, s);
      bl::def_adj_combine(g, scaleP, c->PH, c->RHO, c->ASUM, c->KSUM, c->KAP, st, n > 0, s);
    }
  bl::pi_half(c->gP, c->planP, c->GACC, d, c->PH, s);
  bl::def_out(g, scaleP, c->PH, c->KSUM, vproj, c->Lhat, out, c->flag, s);
}

void op_set_velocity_def(bl_ctx* c, const float2* vraw) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  double* red_reg = c->red + RED_REG * bl::kRedBlocks;
  double* red_data = c->red + RED_DATA * bl::kRedBlocks;
  bl::band_prep(g, vraw, c->bv, 1, c->Lhat64, red_reg, s);
  bl::iota(c->gP, c->planP, c->bv, g.dim, c->VP, s);
  const float2* u1 = def_sweep_forward(c, false);
  bl::iota(g, c->plan, u1, g.dim, c->UG, s);
  bl::def_warp(g, c->UG, c->IG, c->mfinal, c->GP, s);
  bl::energy_partial(g, c->mfinal, c->I1, red_data, s);
  bl::reduce_final2(red_reg, c->scal + S_REG, c->hdev + S_REG, red_data, c->scal + S_DATA,
                    c->hdev + S_DATA, bl::kRedBlocks, s);
  check_launch("set_velocity (deformation)");
  sync(c);
  c->reg = c->hscal[S_REG];
  c->data_sum = c->hscal[S_DATA];
  const double sig = c->prob.sigma;
  c->E = 0.5 * c->reg + c->data_sum / (sig * sig * (double)g.M);
  c->have_v = true;
  c->have_lambda = false;
  if (!std::isfinite(c->E)) throw NonFinite{"energy"};
}

// rho~(1) = pi(Bf) into RHO (Bf = lambda(1) (grad I0) o phi(1) or its incremental form)
void def_terminal_band(bl_ctx* c) {
  const bl::Geo& g = c->g;
  bl::pi_half(g, c->plan, c->Bf, g.dim, c->P, c->stream);
  bl::band_finalize(g, g.dim, nullptr, nullptr, c->P, (float)(1.0 / (double)g.M), c->RHO, c->flag,
                    c->stream, 0);
}

void op_gradient_def(bl_ctx* c, float2* gout) {
  const bl::Geo& g = c->g;
  bl::def_rho1(g, c->mfinal, c->I1, c->GP, c->Bf, c->stream);
  def_terminal_band(c);
  def_sweep_backward(c, c->bv, gout);
  check_launch("gradient (deformation)");
}

void op_hessvec_def(bl_ctx* c, const float2* draw, float2* hout) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  bl::band_prep(g, draw, c->bd, 0, nullptr, nullptr, s);
  bl::iota(c->gP, c->planP, c->bd, g.dim, c->DVP, s);
  const float2* du1 = def_sweep_forward(c, true);
  bl::iota(g, c->plan, du1, g.dim, c->UG, s);
  bl::def_drho1(g, c->UG, c->GP, c->Bf, s);
  def_terminal_band(c);
  def_sweep_backward(c, c->bd, hout);
  check_launch("hessvec (deformation)");
}

// host-mapped mirror of a device scalar slot, for single-problem launches (a batched launch
// publishes nothing to host memory: its scalars are read by the device control kernels)
double* publish(bl_ctx* c, int slot) {
  return (c->g.bat.count > 1 || !c->hdev) ? nullptr : c->hdev + slot;
}

// setup + forward state + energy sums at the raw band vector `vraw` (stationary state
// equation), enqueued only: the regulariser and data sums land in scal[S_REG], scal[S_DATA]
void enqueue_set_velocity(bl_ctx* c, const float2* vraw) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  double* red_reg = c->red + RED_REG * bl::kRedBlocks;
  double* red_data = c->red + RED_DATA * bl::kRedBlocks;
  bl::band_prep(g, vraw, c->bv, 1, c->Lhat64, red_reg, s);
  bl::iota(g, c->plan, c->bv, g.dim + 1, c->V, s);
  timed(c, 6, [&] { bl::setup(g, c->V, c->X, c->YA, s); });
  if (!c->tuned) choose_launch_shapes(c);
  const size_t M = (size_t)g.M;
  for (int n = 0; n < g.nt; ++n)
    timed(c, 0, [&] { bl::state_step(g, c->m + n * M, c->X, c->m + (n + 1) * M, s); });
  // the energy's data term and, in the same pass, the terminal adjoint lambda^Nt into L[nt]
  bl::energy_partial(g, c->m + g.nt * M, c->I1, red_data, s, c->L + g.nt * M);
  c->lamT_valid = true;
  bl::reduce_final2(red_reg, c->scal + S_REG, publish(c, S_REG), red_data, c->scal + S_DATA,
                    publish(c, S_DATA), bl::kRedBlocks, s, false, nullptr, nullptr, g.bat);
  check_launch("set_velocity");
}

// setup + forward state + energy at the raw band vector `vraw` (device, dim components)
void op_set_velocity(bl_ctx* c, const float2* vraw) {
  c->lamT_valid = false;   // set again by the stationary energy pass, which writes lambda^Nt
  if (c->g.deform) {
    op_set_velocity_def(c, vraw);
    return;
  }
  if (c->g.nodes > 1) {
    op_set_velocity_ns(c, vraw);
    return;
  }
  enqueue_set_velocity(c, vraw);
  sync(c);
  finish_set_velocity(c);
}

// E and the state flags from the published sums of enqueue_set_velocity (after a sync)
void finish_set_velocity(bl_ctx* c) {
  const bl::Geo& g = c->g;
  c->reg = c->hscal[S_REG];
  c->data_sum = c->hscal[S_DATA];
  const double sig = c->prob.sigma;
  c->E = 0.5 * c->reg + c->data_sum / (sig * sig * (double)g.M);
  c->have_v = true;
  c->have_lambda = false;
  if (!std::isfinite(c->E)) throw NonFinite{"energy"};
}

// Energy and gradient at the raw band vector `vraw` into gout with one host synchronisation
// (stationary state equation): the energy sums and the non-finite flag of the band outputs
// are published to host-mapped memory and read together; `after` enqueues the caller's
// copies of the results before that synchronisation.
template <class After>
void op_energy_gradient(bl_ctx* c, const float2* vraw, float2* gout, After&& after) {
  enqueue_set_velocity(c, vraw);
  op_gradient(c, gout);
  bl::publish_flag(c->flag, c->hdev + S_FLAG, c->stream);
  after();
  check_launch("energy and gradient");
  sync(c);
  finish_set_velocity(c);
  c->have_lambda = true;   // L holds this velocity's adjoint (the full Newton product reuses it)
  if (c->hscal[S_FLAG] != 0.0) {
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    sync(c);
    throw NonFinite{"gradient"};
  }
}

// backward transport of L[nt] down to L[0], then the body force b = sum_n w_n L[n] grad m^n
// lambda^0 (or dlambda^0) is read by nothing but the body force, which can form it from
// lambda^1 itself: one adjoint launch and the plane's store and reload fewer.  That pays while
// a step's fields stay in the last-level cache (at 128^3 a product takes 513 instead of
// 522 us); on larger grids (Geo::stream_out) the body force then fetches the offsets and
// lambda^1 from HBM at its own, lower rate and loses more than the launch saves (256^3: +104
// us in the body force against 90 us for the adjoint step), so the last step stays separate.
// The full Newton product keeps every stored lambda^n, so a Newton context transports down to
// lambda^0.  Both forms give bitwise the same sums.
bool body_forms_lambda0(const bl::Geo& g) { return !g.newton && !g.stream_out; }

void backward_and_body_force(bl_ctx* c) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M;
  const bool form0 = body_forms_lambda0(g);
  for (int n = g.nt - 1; n >= (form0 ? 1 : 0); --n)
    timed(c, 2, [&] { bl::adj_step(g, c->L + (n + 1) * M, c->YA, c->L + n * M, s); });
  timed(c, 5, [&] { bl::body_force(g, c->L, c->m, c->Bf, s, form0 ? c->YA : nullptr); });
}

// gradient at the current velocity into gout (device, dim components)
bool op_gradient(bl_ctx* c, float2* gout, double* sq_part, double* max_part) {
  if (c->g.deform) {
    op_gradient_def(c, gout);
    return false;
  }
  if (c->g.nodes > 1) {
    op_gradient_ns(c, gout);
    return false;
  }
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M;
  if (!c->lamT_valid) bl::terminal(g, c->m + g.nt * M, c->I1, c->L + g.nt * M, s);
  backward_and_body_force(c);
  c->have_lambda = true;
  bl::pi_half(g, c->plan, c->Bf, g.dim, c->P, s);
  bl::band_finalize(g, g.dim, c->bv, c->Lhat, c->P, (float)(1.0 / (double)g.M), gout, c->flag, s,
                    1, nullptr, nullptr, sq_part, max_part);
  check_launch("gradient");
  return sq_part != nullptr && max_part != nullptr;
}

// Full Newton Hessian-vector product: the Gauss-Newton one plus the incremental adjoint's
// source div(lambda dv) and pi(sum w_n lambda^n grad dm^n); lambda^n (kept in L) comes from the
// gradient at this velocity, or is computed here if no gradient was taken.
void op_hessvec_newton(bl_ctx* c, const float2* draw, float2* hout, double* dot_part) {
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M;
  if (!c->have_lambda) {
    bl::terminal(g, c->m + g.nt * M, c->I1, c->L + g.nt * M, s);
    for (int n = g.nt - 1; n >= 0; --n) bl::adj_step(g, c->L + (n + 1) * M, c->YA, c->L + n * M, s);
    c->have_lambda = true;
  }
  bl::band_prep(g, draw, c->bd, 0, nullptr, nullptr, s);
  bl::iota(g, c->plan, c->bd, g.dim, c->DV, s);
  bl::inc_init(g, c->m, c->DV, c->T0, s);
  float* tin = c->T0;
  float* tout = c->T1;
  for (int n = 0; n + 1 < g.nt; ++n) {
    bl::inc_step_n(g, tin, c->X, c->m + (n + 1) * M, c->DV, tout, c->DM + (n + 1) * M, s);
    std::swap(tin, tout);
  }
  bl::inc_last_n(g, tin, c->X, c->m + g.nt * M, c->DV, c->L + g.nt * M, c->DM + g.nt * M,
                 c->DL + g.nt * M, s);
  const float* uin = c->DL + g.nt * M;   // u^Nt = dlambda^Nt
  float* ua = c->U0;
  float* ub = c->U1;
  for (int n = g.nt - 1; n >= 1; --n) {
    bl::adj_step_n(g, uin, c->YA, c->L + n * M, c->DV, 1, c->DL + n * M, ua, s);
    uin = ua;
    std::swap(ua, ub);
  }
  bl::adj_step_n(g, uin, c->YA, c->L, c->DV, 0, c->DL, nullptr, s);
  bl::body_force_n(g, c->DL, c->m, c->L, c->DM, c->Bf, s);
  bl::pi_half(g, c->plan, c->Bf, g.dim, c->P, s);
  bl::band_finalize(g, g.dim, c->bd, c->Lhat, c->P, (float)(1.0 / (double)g.M), hout, c->flag, s,
                    1, draw, dot_part);
  check_launch("hessvec (Newton)");
}

// Gauss-Newton Hessian-vector product of the raw direction draw into hout
bool op_hessvec(bl_ctx* c, const float2* draw, float2* hout, double* dot_part) {
  if (c->g.deform) {
    op_hessvec_def(c, draw, hout);
    return false;
  }
  if (c->g.nodes > 1) {
    op_hessvec_ns(c, draw, hout);
    return false;
  }
  if (c->g.newton) {
    op_hessvec_newton(c, draw, hout, dot_part);
    return dot_part != nullptr;
  }
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const size_t M = (size_t)g.M;
  bl::band_prep(g, draw, c->bd, 0, nullptr, nullptr, s);
  bl::iota_xy(g, c->plan, c->bd, g.dim, s);
  timed(c, 3, [&] { bl::iota_z(g, c->plan, g.dim, c->DV, s); });
  bl::inc_init(g, c->m, c->DV, c->T0, s);
  float* tin = c->T0;
  float* tout = c->T1;
  for (int n = 0; n + 1 < g.nt; ++n) {
    timed(c, 1, [&] { bl::inc_step(g, tin, c->X, c->m + (n + 1) * M, c->DV, tout, s); });
    std::swap(tin, tout);
  }
  bl::inc_last(g, tin, c->X, c->m + g.nt * M, c->DV, c->L + g.nt * M, s);
  c->lamT_valid = false;   // L[nt] holds the incremental terminal adjoint now
  backward_and_body_force(c);
  timed(c, 4, [&] { bl::pi_z(g, c->plan, c->Bf, g.dim, s); });
  bl::pi_yx(g, c->plan, g.dim, c->P, s);
  bl::band_finalize(g, g.dim, c->bd, c->Lhat, c->P, (float)(1.0 / (double)g.M), hout, c->flag, s,
                    1, draw, dot_part);
  check_launch("hessvec");
  return dot_part != nullptr;
}

void check_flag(bl_ctx* c, const char* what) {
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (h) {
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    sync(c);
    throw NonFinite{what};
  }
}

// <g, g>, max |g| and the non-finite flag of the last band kernels, in one synchronisation
// <a, b> over a velocity-shaped band vector into partials pa: the plain l2 product, or for a
// non-stationary velocity the trapezoid-weighted one
void vec_dot_partial(bl_ctx* c, const float2* a, const float2* b, double* pa) {
  const bl::Geo& g = c->g;
  if (g.nodes > 1) bl::dot_partial_w(g, a, b, pa, c->stream);
  else bl::dot_partial(a, b, (int64_t)g.dim * g.B, pa, c->stream, g.bat);
}

// the projected velocity (first dim of the dim + 1 components per node in bv) into dst
void copy_projected_velocity(bl_ctx* c, float2* dst) {
  const bl::Geo& g = c->g;
  const size_t B = (size_t)g.B;
  for (int n = 0; n < g.nodes; ++n)
    HIP_TRY(hipMemcpyAsync(dst + (size_t)n * g.dim * B, c->bv + (size_t)n * (g.dim + 1) * B,
                           band_bytes(g) * g.dim, hipMemcpyDeviceToDevice, c->stream));
}

// |g|^2 and max |g| of gvec (published) with the non-finite flag; have_partials: the gradient's
// band finalisation already wrote their partials to RED_A / RED_B
void grad_stats(bl_ctx* c, const float2* gvec, double* gg, double* ginf, bool have_partials) {
  const int64_t n = (int64_t)c->g.nodes * c->g.dim * c->g.B;
  double* pa = c->red + RED_A * bl::kRedBlocks;
  double* pb = c->red + RED_B * bl::kRedBlocks;
  if (!have_partials) {
    vec_dot_partial(c, gvec, gvec, pa);
    bl::maxabs_partial(gvec, n, pb, c->stream);
  }
  bl::reduce_final2(pa, c->scal + S_GG, c->hdev + S_GG, pb, c->scal + S_GINF, c->hdev + S_GINF,
                    have_partials ? bl::finalize_blocks(c->g) : bl::kRedBlocks, c->stream, true,
                    c->flag, c->hdev + S_FLAG);
  check_launch("gradient norms");
  sync(c);
  if (c->hscal[S_FLAG] != 0.0) {
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    sync(c);
    throw NonFinite{"gradient"};
  }
  *gg = c->hscal[S_GG];
  *ginf = c->hscal[S_GINF];
}

// enqueue z = r / Lhat with <r, r> -> slot S_RR (also published) and <r, z> -> slot rz_slot
void enqueue_precond(bl_ctx* c, int rz_slot) {
  double* pa = c->red + RED_A * bl::kRedBlocks;
  double* pb = c->red + RED_B * bl::kRedBlocks;
  bl::precond_dots(c->g, c->sr, c->Lhat, c->sz, pa, pb, c->stream);
  bl::reduce_final2(pa, c->scal + S_RR, c->hdev + S_RR, pb, c->scal + rz_slot, nullptr,
                    bl::kRedBlocks, c->stream);
}

double dev_sqdiff(bl_ctx* c, const float* a, const float* b) {
  double* part = c->red + RED_A * bl::kRedBlocks;
  bl::sqdiff_partial(a, b, c->g.M, part, c->stream);
  bl::reduce_final(part, bl::kRedBlocks, c->scal + S_SQD, c->stream, c->hdev + S_SQD);
  check_launch("sqdiff");
  sync(c);
  return c->hscal[S_SQD];
}

void load_images(bl_ctx* c, const float* I0, const float* I1) {
  const size_t pb = plane_bytes(c->g);
  HIP_TRY(hipMemcpyAsync(c->m, I0, pb, in_kind(c), c->stream));
  if (I1) HIP_TRY(hipMemcpyAsync(c->I1, I1, pb, in_kind(c), c->stream));
  else HIP_TRY(hipMemsetAsync(c->I1, 0, pb, c->stream));
  if (c->IG) {
    bl::def_ig4(c->g, c->m, c->IG, c->stream);
    check_launch("image gradient");
  }
}

void load_band(bl_ctx* c, const float* src, float2* dst, int ncomp) {
  HIP_TRY(hipMemcpyAsync(dst, src, band_bytes(c->g) * ncomp, in_kind(c), c->stream));
}
void store_band(bl_ctx* c, const float2* src, float* dst, int ncomp) {
  HIP_TRY(hipMemcpyAsync(dst, src, band_bytes(c->g) * ncomp,
                         c->devptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
}
void store_plane(bl_ctx* c, const float* src, float* dst, size_t nplanes) {
  HIP_TRY(hipMemcpyAsync(dst, src, plane_bytes(c->g) * nplanes,
                         c->devptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
}

// ------------------------------------------------------------------------------ solver
void fill_default(bl_solver_opts* o) {
  o->max_gn = 10;
  o->max_pcg = 10;
  o->gtol = 1e-3;
  o->c1 = 1e-4;
  o->max_halvings = 10;
}

// Gauss-Newton-Krylov on the device vectors of the context (reading R-LS / R-PCG):
// sv holds the initial guess on entry and the result on exit.
void solve(bl_ctx* c, const bl_solver_opts& o, bl_stats* st) {
  // Scalars stay on the device wherever only kernels consume them (the PCG step length and
  // direction update); the host synchronises once per PCG step for its stopping test, once per
  // line-search trial for E, and once per gradient for its norms and the non-finite flag.
  const bl::Geo& g = c->g;
  hipStream_t s = c->stream;
  const int64_t nb = (int64_t)g.nodes * g.dim * g.B;
  double* pa = c->red + RED_A * bl::kRedBlocks;
  double* pb = c->red + RED_B * bl::kRedBlocks;
  double* pc = c->red + RED_C * bl::kRedBlocks;
  const double den = dev_sqdiff(c, c->m, c->I1);  // |I0 - I1|^2
  auto mse = [&]() { return den > 0 ? 100.0 * c->data_sum / den : 0.0; };

  op_set_velocity(c, c->sv);
  copy_projected_velocity(c, c->sv);
  double gg, ginf0;
  grad_stats(c, c->sg, &gg, &ginf0, op_gradient(c, c->sg, pa, pb));
  double E = c->E;
  const double g0n = std::sqrt(std::max(gg, 0.0));
  st->E[0] = E;
  st->mse_rel[0] = mse();
  st->ginf_rel[0] = 1.0;
  st->gradients = 1;
  st->evaluations = 1;
  st->status = BL_MAXITER;
  if (ginf0 == 0.0) {
    st->status = BL_CONVERGED;
    st->ginf_rel[0] = 0.0;
    return;
  }
  double ginf = ginf0;
  for (int it = 0; it < o.max_gn; ++it) {
    if (ginf / ginf0 < o.gtol) {
      st->status = BL_CONVERGED;
      break;
    }
    const double gn = std::sqrt(std::max(gg, 0.0));
    const double eta = std::min(0.5, std::sqrt(gn / g0n));
    const double thr = eta * gn;
    const double thr2 = thr * thr;
    // PCG on H delta = -g with preconditioner K = 1/Lhat, delta_0 = 0
    HIP_TRY(hipMemsetAsync(c->sdelta, 0, nb * sizeof(float2), s));
    HIP_TRY(hipMemsetAsync(c->sr, 0, nb * sizeof(float2), s));
    bl::axpy(c->sr, c->sg, -1.0, nb, s);  // r = -g
    int rz_cur = S_RZ0, rz_next = S_RZ1;
    enqueue_precond(c, rz_cur);
    HIP_TRY(hipMemcpyAsync(c->sp, c->sz, nb * sizeof(float2), hipMemcpyDeviceToDevice, s));
    int iters = 0;
    for (int j = 0; j < o.max_pcg; ++j) {
      // the partials of <p, Hp> come with the product's last kernel where it can form them
      const bool fused = op_hessvec(c, c->sp, c->sHp, pc);
      st->hessvecs += 1;
      if (!fused) vec_dot_partial(c, c->sp, c->sHp, pc);
      // <p, Hp>, alpha = <r, z> / <p, Hp>, zero when <p, Hp> <= 0 (then neither vector moves);
      // delta, r, z = K r and the partials of <r, r>, <r, z> in one launch
      bl::pcg_step(g, c->sp, c->sHp, c->scal + rz_cur, pc,
                   fused ? bl::finalize_blocks(g) : bl::kRedBlocks, c->scal + S_PHP,
                   c->hdev + S_PHP, c->sdelta, c->sr, c->Lhat, c->sz, pa, pb, s);
      bl::reduce_final2(pa, c->scal + S_RR, c->hdev + S_RR, pb, c->scal + rz_next, nullptr,
                        bl::kRedBlocks, s);
      check_launch("pcg");
      sync(c);
      const double pHp = c->hscal[S_PHP];
      if (!(pHp > 0.0)) {
        if (iters == 0)  // z = K r of the unchanged r: the preconditioned steepest-descent step
          HIP_TRY(hipMemcpyAsync(c->sdelta, c->sz, nb * sizeof(float2), hipMemcpyDeviceToDevice, s));
        break;
      }
      iters += 1;
      // |r| <= eta |g|, compared as squares (the same FP64 operations as the batched engine's
      // device-side test, so both take the same decisions)
      if (std::max(c->hscal[S_RR], 0.0) <= thr2) break;
      bl::xpby_dev(c->sp, c->sz, c->scal + rz_next, c->scal + rz_cur, nb, s);  // p = z + beta p
      std::swap(rz_cur, rz_next);
    }
    check_launch("pcg");
    st->pcg_iters[it] = iters;
    st->pcg_total += iters;
    // Armijo backtracking on E along delta; the slope <g, delta> arrives with the first trial
    vec_dot_partial(c, c->sg, c->sdelta, pa);
    bl::reduce_final(pa, bl::kRedBlocks, c->scal + S_SLOPE, s, c->hdev + S_SLOPE);
    double eps = 1.0;
    bool accepted = false;
    int trials = 0;
    for (int t = 0; t <= o.max_halvings; ++t) {
      trials += 1;
      bl::add_scaled(c->stry, c->sv, c->sdelta, eps, nb, s);
      op_set_velocity(c, c->stry);
      st->evaluations += 1;
      const double slope = c->hscal[S_SLOPE];
      if (c->E <= E + o.c1 * eps * slope) {
        accepted = true;
        break;
      }
      eps *= 0.5;
    }
    st->ls_trials[it] = trials;
    if (!accepted) {
      st->status = BL_STALLED;
      st->eps[it] = 0.0;
      op_set_velocity(c, c->sv);  // state of the returned velocity
      break;
    }
    st->eps[it] = eps;
    copy_projected_velocity(c, c->sv);
    E = c->E;
    grad_stats(c, c->sg, &gg, &ginf, op_gradient(c, c->sg, pa, pb));
    st->gradients += 1;
    st->gn_iters += 1;
    st->E[st->gn_iters] = E;
    st->mse_rel[st->gn_iters] = mse();
    st->ginf_rel[st->gn_iters] = ginf / ginf0;
    if (it + 1 == o.max_gn && ginf / ginf0 < o.gtol) st->status = BL_CONVERGED;
  }
}

size_t ctx_bytes(const bl::Geo& g, bool transport, bool solver, bool mixed) {
  return plan_layout(g, transport, solver, mixed).total;
}

// ---------------------------------------------------------------- idle context cache
// The one-shot calls (register, gradient, H v, warp) take an idle context of the same problem
// on the same device if one is cached and hand it back after a successful call (their work is
// complete then: each ends with a host synchronisation), so repeated calls on one problem
// shape allocate no device memory and rebuild no tables.  At most kCacheMax idle contexts and
// kCacheBytes of device memory are kept; bl_lddmm_release_cached frees them.
constexpr size_t kCacheMax = 8;
constexpr size_t kCacheBytes = size_t(32) << 30;
std::mutex g_cache_mu;
std::vector<bl_ctx*> g_idle;   // oldest first

bool same_problem(const bl_ctx* c, const bl_problem* p, int device, bool solver) {
  const bl_problem& q = c->prob;
  if (c->device != device || !c->transport || (c->sv != nullptr) != solver) return false;
  if (q.dim != p->dim || q.nt != p->nt || q.s != p->s || q.gamma != p->gamma ||
      q.precision != p->precision || q.flags != p->flags)
    return false;
  for (int j = 0; j < 3; ++j)
    if (q.n[j] != p->n[j] || q.k[j] != p->k[j]) return false;
  return q.alpha == p->alpha && q.sigma == p->sigma;
}

void free_idle(std::vector<bl_ctx*>& v) {
  int dev = 0;
  const bool have_dev = hipGetDevice(&dev) == hipSuccess;
  for (bl_ctx* c : v) destroy_ctx(c);   // switches to each context's device
  v.clear();
  if (have_dev) (void)hipSetDevice(dev);
}

struct CachedCtx {
  bl_ctx* c = nullptr;
  bool ok = false;
  CachedCtx(const bl_problem* prob, const bl::Geo& g, bool solver) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      for (size_t i = 0; i < g_idle.size(); ++i)
        if (same_problem(g_idle[i], prob, dev, solver)) {
          c = g_idle[i];
          g_idle.erase(g_idle.begin() + i);
          break;
        }
    }
    if (c) {
      if (c->devptr) c->stream = (hipStream_t)prob->stream;
      c->have_v = false;
      return;
    }
    try {
      c = create_ctx(prob, g, true, solver);
    } catch (const std::bad_alloc&) {
      // idle cached contexts may hold the memory: free them and try once more
      std::vector<bl_ctx*> drop;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        drop.swap(g_idle);
      }
      free_idle(drop);
      c = create_ctx(prob, g, true, solver);
    }
  }
  ~CachedCtx() {
    if (!c) return;
    if (!ok) {
      destroy_ctx(c);
      return;
    }
    if (c->timing) {
      for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
      c->ev_pool.clear();
      c->ev_used.clear();
      c->ev_pairs.clear();
      c->ev_next = 0;
      c->timing = false;
    }
    if (c->devptr) c->stream = nullptr;   // the caller's stream is not kept
    std::vector<bl_ctx*> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_idle.push_back(c);
      size_t bytes = 0;
      for (bl_ctx* x : g_idle) bytes += x->arena_bytes;
      while (g_idle.size() > kCacheMax || (bytes > kCacheBytes && g_idle.size() > 1)) {
        bytes -= g_idle.front()->arena_bytes;
        drop.push_back(g_idle.front());
        g_idle.erase(g_idle.begin());
      }
    }
    free_idle(drop);
  }
};

}  // namespace host
}  // namespace bl

// ================================================================================ C-ABI
using namespace bl::host;

extern "C" {

void bl_lddmm_default_opts(bl_solver_opts* opts) {
  if (opts) fill_default(opts);
}

const char* bl_lddmm_last_error(void) { return t_err.c_str(); }

int bl_lddmm_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

void bl_lddmm_tune_reload(void) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_shapes.clear();
  read_shape_file();
}

void bl_lddmm_release_cached(void) {
  std::vector<bl_ctx*> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    drop.swap(g_idle);
  }
  free_idle(drop);
}

uint64_t bl_lddmm_footprint(const bl_problem* prob) {
  bl::Geo g;
  if (validate(prob, &g) != BL_OK) return 0;
  return (uint64_t)plan_layout(g, true, true, prob->precision == BL_MIXED).total;
}

int bl_lddmm_ctx_create(const bl_problem* prob, const float* I0, const float* I1, bl_ctx** out) {
  t_err.clear();
  if (out) *out = nullptr;
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (!out || !I0 || !I1) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CtxHolder h;
    h.c = create_ctx(prob, g, true, true);
    load_images(h.c, I0, I1);
    sync(h.c);
    *out = h.c;
    h.c = nullptr;
    return BL_OK;
  });
}

void bl_lddmm_ctx_destroy(bl_ctx* ctx) { destroy_ctx(ctx); }

int bl_lddmm_ctx_set_velocity(bl_ctx* c, const float* v_hat, double* energy, float* g_hat) {
  t_err.clear();
  if (!c || !v_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    HIP_TRY(hipSetDevice(c->device));
    load_band(c, v_hat, c->braw, c->g.nodes * c->g.dim);
    if (g_hat && !c->g.deform && c->g.nodes == 1) {
      op_energy_gradient(c, c->braw, c->bout,
                         [&]() { store_band(c, c->bout, g_hat, c->g.dim); });
      if (energy) *energy = c->E;
      t_collect(c);
      return BL_OK;
    }
    op_set_velocity(c, c->braw);
    if (energy) *energy = c->E;
    if (g_hat) {
      op_gradient(c, c->bout);
      store_band(c, c->bout, g_hat, c->g.nodes * c->g.dim);
      check_flag(c, "gradient");
    }
    t_collect(c);
    return BL_OK;
  });
}

int bl_lddmm_ctx_hessvec(bl_ctx* c, const float* dv_hat, float* hv_hat) {
  t_err.clear();
  if (!c || !dv_hat || !hv_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  if (!c->have_v) return fail(BL_E_INVALID, "no velocity set on this context");
  return guarded([&]() {
    HIP_TRY(hipSetDevice(c->device));
    if (c->devptr) {
      op_hessvec(c, reinterpret_cast<const float2*>(dv_hat), reinterpret_cast<float2*>(hv_hat));
      return BL_OK;
    }
    load_band(c, dv_hat, c->braw, c->g.nodes * c->g.dim);
    op_hessvec(c, c->braw, c->bout);
    store_band(c, c->bout, hv_hat, c->g.nodes * c->g.dim);
    check_flag(c, "Hessian-vector product");
    t_collect(c);
    return BL_OK;
  });
}

int bl_lddmm_ctx_get_field(bl_ctx* c, int32_t which, int32_t index, float* out) {
  t_err.clear();
  if (!c || !out) return fail(BL_E_INVALID, "NULL pointer argument");
  const bl::Geo& g = c->g;
  const float* src = nullptr;
  const float4* packed = nullptr;
  int comp = 0;
  const size_t M = (size_t)g.M;
  switch (which) {
    case BL_FIELD_VELOCITY: if (index >= 0 && index < g.dim) src = c->V + index * M; break;
    case BL_FIELD_DIV: if (index == 0) src = c->V + g.dim * M; break;
    case BL_FIELD_X: if (index >= 0 && index < g.dim) src = c->X + index * M; break;
    case BL_FIELD_Y: if (index >= 0 && index < g.dim) { packed = c->YA; comp = index; } break;
    case BL_FIELD_A: if (index == 0) { packed = c->YA; comp = 3; } break;
    case BL_FIELD_STATE: if (index >= 0 && index <= g.nt) src = c->m + index * M; break;
    default: break;
  }
  if (g.deform) {   // only I0 and m(1) are grid fields of the deformation method
    src = nullptr;
    packed = nullptr;
    if (which == BL_FIELD_STATE && index == 0) src = c->m;
    if (which == BL_FIELD_STATE && index == g.nt) src = c->mfinal;
  }
  if (!src && !packed) return fail(BL_E_INVALID, "unknown field or index out of range");
  if (!c->have_v && which != BL_FIELD_STATE) return fail(BL_E_INVALID, "no velocity set on this context");
  return guarded([&]() {
    HIP_TRY(hipSetDevice(c->device));
    if (packed) {
      bl::unpack4(g, comp, packed, c->T0, c->stream);   // T0 is free between operations
      check_launch("get_field");
      src = c->T0;
    }
    store_plane(c, src, out, 1);
    sync(c);
    return BL_OK;
  });
}

int bl_lddmm_gradient(const bl_problem* prob, const float* I0, const float* I1,
                      const float* v_hat, float* g_hat, double* energy) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (!I0 || !I1 || !v_hat || !g_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CachedCtx h(prob, g, false);
    load_images(h.c, I0, I1);
    load_band(h.c, v_hat, h.c->braw, g.nodes * g.dim);
    if (!g.deform && g.nodes == 1) {
      op_energy_gradient(h.c, h.c->braw, h.c->bout,
                         [&]() { store_band(h.c, h.c->bout, g_hat, g.dim); });
    } else {
      op_set_velocity(h.c, h.c->braw);
      op_gradient(h.c, h.c->bout);
      store_band(h.c, h.c->bout, g_hat, g.nodes * g.dim);
      check_flag(h.c, "gradient");
    }
    if (energy) *energy = h.c->E;
    h.ok = true;
    return BL_OK;
  });
}

int bl_lddmm_hessvec(const bl_problem* prob, const float* I0, const float* I1,
                     const float* v_hat, const float* dv_hat, float* hv_hat) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (!I0 || !I1 || !v_hat || !dv_hat || !hv_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CachedCtx h(prob, g, false);
    load_images(h.c, I0, I1);
    load_band(h.c, v_hat, h.c->braw, g.nodes * g.dim);
    op_set_velocity(h.c, h.c->braw);
    load_band(h.c, dv_hat, h.c->braw, g.nodes * g.dim);
    op_hessvec(h.c, h.c->braw, h.c->bout);
    store_band(h.c, h.c->bout, hv_hat, g.nodes * g.dim);
    check_flag(h.c, "Hessian-vector product");
    h.ok = true;
    return BL_OK;
  });
}

int bl_lddmm_warp(const bl_problem* prob, const float* I0, const float* v_hat, float* warped) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (!I0 || !v_hat || !warped) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CachedCtx h(prob, g, false);
    load_images(h.c, I0, nullptr);
    load_band(h.c, v_hat, h.c->braw, g.nodes * g.dim);
    op_set_velocity(h.c, h.c->braw);
    store_plane(h.c, h.c->mfinal, warped, 1);
    sync(h.c);
    h.ok = true;
    return BL_OK;
  });
}

int bl_lddmm_register(const bl_problem* prob, const bl_solver_opts* opts, const float* I0,
                      const float* I1, float* v_hat, float* warped, bl_stats* stats) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (int r = validate_opts(opts)) return r;
  if (!I0 || !I1 || !v_hat) return fail(BL_E_INVALID, "NULL pointer argument");
  bl_solver_opts o;
  if (opts) o = *opts; else fill_default(&o);
  return guarded([&]() {
    const auto t0 = std::chrono::steady_clock::now();
    bl_stats local;
    std::memset(&local, 0, sizeof(local));
    CachedCtx h(prob, g, true);
    load_images(h.c, I0, I1);
    load_band(h.c, v_hat, h.c->sv, g.nodes * g.dim);
    solve(h.c, o, &local);
    store_band(h.c, h.c->sv, v_hat, g.nodes * g.dim);
    if (warped) store_plane(h.c, h.c->mfinal, warped, 1);
    sync(h.c);
    local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = local;
    h.ok = true;
    return BL_OK;
  });
}

int bl_band_to_grid(const bl_problem* prob, int32_t ncomp, const float* band, float* grid) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (ncomp < 1 || ncomp > 4) return fail(BL_E_INVALID, "ncomp must be in [1, 4]");
  if (!band || !grid) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CtxHolder h;
    h.c = create_ctx(prob, g, false, false);
    bl_ctx* c = h.c;
    // project each component separately through the prep kernel (it handles dim components)
    bl::Geo g1 = g;
    g1.dim = 1;
    g1.gamma = 0;   // single components: Hermitian projection only
    for (int i = 0; i < ncomp; ++i) {
      load_band(c, band + (size_t)2 * g.B * i, c->braw, 1);
      bl::band_prep(g1, c->braw, c->bv + (size_t)g.B * i, 0, nullptr, nullptr, c->stream);
    }
    bl::iota(g, c->plan, c->bv, ncomp, c->V, c->stream);
    check_launch("band_to_grid");
    store_plane(c, c->V, grid, ncomp);
    sync(c);
    return BL_OK;
  });
}

int bl_grid_to_band(const bl_problem* prob, int32_t ncomp, const float* grid, float* band) {
  t_err.clear();
  bl::Geo g;
  if (int r = validate(prob, &g)) return r;
  if (ncomp < 1 || ncomp > 4) return fail(BL_E_INVALID, "ncomp must be in [1, 4]");
  if (!band || !grid) return fail(BL_E_INVALID, "NULL pointer argument");
  return guarded([&]() {
    CtxHolder h;
    h.c = create_ctx(prob, g, false, false);
    bl_ctx* c = h.c;
    HIP_TRY(hipMemcpyAsync(c->V, grid, plane_bytes(g) * ncomp, in_kind(c), c->stream));
    bl::pi_half(g, c->plan, c->V, ncomp, c->P, c->stream);
    bl::band_finalize(g, ncomp, nullptr, c->Lhat, c->P, (float)(1.0 / (double)g.M), c->bout,
                      c->flag, c->stream);
    check_launch("grid_to_band");
    store_band(c, c->bout, band, ncomp);
    sync(c);
    return BL_OK;
  });
}

int bl_lddmm_ctx_launch_shapes(bl_ctx* c, int32_t zv_out[4]) {
  t_err.clear();
  if (!c || !zv_out) return fail(BL_E_INVALID, "NULL pointer argument");
  for (int k = 0; k < 4; ++k) zv_out[k] = c->g.dim == 3 ? c->g.zv[k] : 1;
  return BL_OK;
}

int bl_kernel_timing_enable(bl_ctx* c, int32_t on) {
  t_err.clear();
  if (!c) return fail(BL_E_INVALID, "NULL context");
  return guarded([&]() {
    HIP_TRY(hipSetDevice(c->device));
    if (on && c->ev_pool.empty()) {
      c->ev_pool.resize(8192);
      c->ev_pairs.resize(4096);
      for (auto& e : c->ev_pool) HIP_TRY(hipEventCreate(&e));
    }
    t_collect(c);
    c->timing = on != 0;
    return BL_OK;
  });
}

int bl_kernel_timing_read(bl_ctx* c, int32_t kclass, int64_t* launches, double* ms) {
  t_err.clear();
  if (!c || !launches || !ms) return fail(BL_E_INVALID, "NULL pointer argument");
  if (kclass < 0 || kclass > 6) return fail(BL_E_INVALID, "kernel class must be in [0, 6]");
  return guarded([&]() {
    HIP_TRY(hipSetDevice(c->device));
    t_collect(c);
    *launches = c->t_launch[kclass];
    *ms = c->t_ms[kclass];
    c->t_launch[kclass] = 0;
    c->t_ms[kclass] = 0;
    return BL_OK;
  });
}

}  // extern "C"
