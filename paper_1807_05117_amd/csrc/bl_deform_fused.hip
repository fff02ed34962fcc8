// Fused stage kernels of the deformation state equation on the product grid (3D).
//
// One Runge-Kutta stage (or one stage of the transposed sweep) is three launches instead of a
// chain of separate transform, product and band kernels:
//   1. xy:  band (kz >= 0 half) -> F2[c][h][y][x]: the x and y contractions of iota for one
//           (component, h) plane and a chunk of x, the band plane staged in LDS.  In the
//           derivative form the components are the spectral derivatives d~_j U_i (c = i dim + j)
//           formed on the fly from the state U.
//   2. col: per (y, x) column of the product grid: the z contraction of iota, the pointwise
//           products (and their side outputs), and the z contraction of pi, the column's z
//           values exchanged through LDS; two lanes per column split the kz spectrum.
//   3. yx:  G[c][h][y][x] -> the band: the x and y contractions of pi for one (component, h)
//           plane and a chunk of kx, the G plane staged in LDS (the transposed sweep stages
//           its three derivative planes together), followed by the band-side update of the
//           stage (forward) or of the transposed sweep (backward) at kz = h and at the
//           conjugate-mirror index -k.  On the kz = 0 plane the entry k is owned by the half
//           ky > 0 or (ky = 0, kx >= 0); its owner writes k and -k, so the result is exactly
//           Hermitian, and k = 0 takes the real part.
// Twiddle tables are those of the product grid's transform plan (bl_dft.hip layout).
// These kernels are bound by memory latency at ~1.5 waves per SIMD, so every global load a
// phase needs is issued before its first wait: no load sits behind a condition (a guarded load
// compiles to a branch and a wait) and no runtime loop alternates loads and LDS stores.
#include "bl_internal.h"

#include <mutex>

namespace bl {
namespace {

constexpr int kColW = 32;     // columns per column-kernel block (two lanes each)
constexpr int kColWaves = 8;  // waves per column-kernel block
constexpr int kXC = 16;       // x outputs per iota xy block
constexpr int kKC = 4;        // kx outputs per pi yx block

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}
// acc += a * conj(b)
__device__ __forceinline__ void cmac_conj(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.y, b.x, acc.y);
  acc.y = fmaf(-a.x, b.y, acc.y);
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// q = 2 pi k / l of band index j on axis a (l from the image grid)
__device__ __forceinline__ float qaxis(const Geo& g, int a, int j) {
  const float two_pi = 6.283185307179586f;
  const int kv = a == 0 ? j - g.kx / 2 : (a == 1 ? j - g.ky / 2 : j - g.kz0);
  const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
  return two_pi * (float)kv * ((float)g.nref / (float)n);
}

// Staging of tables into LDS with a thread's loads in flight together.  A runtime loop of
// load-then-store waits for one memory round trip per iteration; here a thread first loads R
// entries of a table into registers (entries past the end read the clamped last entry), and
// only then stores them.  Loads of several tables are issued before any of their stores.
template <int NT, int R>
struct Stager {
  float2 v[R];
  template <class Ld>
  __device__ __forceinline__ void load(int n, int base, Ld ld) {
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = ld(min(base + (int)threadIdx.x + NT * u, n - 1));
  }
  template <class St>
  __device__ __forceinline__ void store(int n, int base, St st) const {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int o = base + (int)threadIdx.x + NT * u;
      if (o < n) st(o, v[u]);
    }
  }
};

// ---------------------------------------------------------------------------- 1. iota xy
// block (c * kzh + h, x chunk); F2[c][h][y][x] = sum_ky sum_kx S[ky][kx] Tx[kx][x] Ty[ky][y]
// with S the band plane kz = h of component c (deriv: i q_j U_i for c = i dim + j).  The band
// plane and the twiddles the block needs are staged in LDS first (all loads in flight at once).
__global__ __launch_bounds__(256) void k_fx_iota_xy(Geo g, Geo gp, const float2* __restrict__ in,
                                                    int deriv, const float2* __restrict__ tw_x,
                                                    const float2* __restrict__ tw_y, int nyp,
                                                    float2* __restrict__ F2) {
  extern __shared__ float2 lds[];
  const int KX = g.kx, KY = g.ky, PX = gp.nx, PY = gp.ny;
  const int SX = KX + 1;                // padded row: rows fall in different LDS banks
  float2* S = lds;                      // [KY][SX]
  float2* T = S + (size_t)KY * SX;      // [KY][kXC]
  float2* Txc = T + (size_t)KY * kXC;   // [KX][kXC]
  float2* Ty = Txc + (size_t)KX * kXC;  // [KY][PY]
  const int ch = blockIdx.x;
  const int c = ch / g.kzh, h = ch - c * g.kzh;
  const int x0 = blockIdx.y * kXC;
  const int jz = g.kz0 + h;
  const int d = g.dim;
  const int ci = deriv ? c / d : c;
  const int cj = deriv ? c - ci * d : 0;
  const float2* plane = in + ((size_t)ci * g.kz + jz) * KY * KX;
  // the band plane and both twiddle tables, all loads of a round in flight together (one round
  // up to a 32 x 32 band and 48 y values)
  const int nS = KY * KX, nX = KX * kXC, nY = KY * PY;
  const int rounds = max(max((nS + 1023) / 1024, (nX + 511) / 512), (nY + 1535) / 1536);
  for (int r = 0; r < rounds; ++r) {
    Stager<256, 4> sS;
    Stager<256, 2> sX;
    Stager<256, 6> sY;
    sS.load(nS, r * 1024, [&](int o) { return plane[o]; });
    sX.load(nX, r * 512, [&](int o) {
      const int jx = o / kXC, xl = o - jx * kXC;
      return tw_x[(size_t)jx * PX + min(x0 + xl, PX - 1)];
    });
    sY.load(nY, r * 1536, [&](int o) {
      const int jy = o / PY, y = o - jy * PY;
      return tw_y[(size_t)jy * nyp + y];
    });
    sS.store(nS, r * 1024, [&](int o, float2 v) {
      const int jy = o / KX, jx = o - jy * KX;
      if (deriv) {
        const float q = cj == 0 ? qaxis(g, 0, jx) : (cj == 1 ? qaxis(g, 1, jy) : qaxis(g, 2, jz));
        v = make_float2(-q * v.y, q * v.x);
      }
      S[jy * SX + jx] = v;
    });
    sX.store(nX, r * 512, [&](int o, float2 v) { Txc[o] = v; });
    sY.store(nY, r * 1536, [&](int o, float2 v) { Ty[o] = v; });
  }
  __syncthreads();
  // Both passes give a thread several outputs of one column xl (256 is a multiple of kXC) and
  // compute them together: the operand they share is read once per term, and their chains of
  // dependent LDS reads run side by side.  Each output keeps its own two alternating partial
  // sums, as a single-output loop would.
  const int xl = threadIdx.x % kXC;
  // x: T[jy][xl] = sum_jx S[jy][jx] Tx[jx][x0 + xl], two rows per thread and round
  const int nT = KY * kXC;
  for (int ob = 0; ob < nT; ob += 512) {
    const int o0 = ob + threadIdx.x, o1 = o0 + 256;
    const int jy0 = min(o0, nT - 1) / kXC, jy1 = min(o1, nT - 1) / kXC;
    float2 a0 = make_float2(0.f, 0.f), b0 = a0, a1 = a0, b1 = a0;
    int jx = 0;
#pragma unroll 4
    for (; jx + 1 < KX; jx += 2) {
      const float2 t0 = Txc[jx * kXC + xl], t1 = Txc[(jx + 1) * kXC + xl];
      cmac(a0, S[jy0 * SX + jx], t0);
      cmac(b0, S[jy0 * SX + jx + 1], t1);
      cmac(a1, S[jy1 * SX + jx], t0);
      cmac(b1, S[jy1 * SX + jx + 1], t1);
    }
    if (jx < KX) {
      const float2 t0 = Txc[jx * kXC + xl];
      cmac(a0, S[jy0 * SX + jx], t0);
      cmac(a1, S[jy1 * SX + jx], t0);
    }
    if (o0 < nT) T[o0] = make_float2(a0.x + b0.x, a0.y + b0.y);
    if (o1 < nT) T[o1] = make_float2(a1.x + b1.x, a1.y + b1.y);
  }
  __syncthreads();
  // y: F2[y][x0 + xl] = sum_jy T[jy][xl] Ty[jy][y], three rows per thread and round
  float2* dst = F2 + (size_t)ch * PY * PX;
  const int nF = PY * kXC;
  const bool xin = x0 + xl < PX;
  for (int ob = 0; ob < nF; ob += 768) {
    int yr[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) yr[u] = min(ob + (int)threadIdx.x + 256 * u, nF - 1) / kXC;
    float2 a[3], b[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) a[u] = b[u] = make_float2(0.f, 0.f);
    int jy = 0;
#pragma unroll 2
    for (; jy + 1 < KY; jy += 2) {
      const float2 t0 = T[jy * kXC + xl], t1 = T[(jy + 1) * kXC + xl];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        cmac(a[u], t0, Ty[jy * PY + yr[u]]);
        cmac(b[u], t1, Ty[(jy + 1) * PY + yr[u]]);
      }
    }
    if (jy < KY) {
      const float2 t0 = T[jy * kXC + xl];
#pragma unroll
      for (int u = 0; u < 3; ++u) cmac(a[u], t0, Ty[jy * PY + yr[u]]);
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int o = ob + (int)threadIdx.x + 256 * u;
      if (xin && o < nF)
        dst[(size_t)yr[u] * PX + x0 + xl] = make_float2(a[u].x + b[u].x, a[u].y + b[u].y);
    }
  }
}

// ---------------------------------------------------------------------------- 2. columns
// Block (32 columns, component), eight waves: lane l of a wave serves column l mod 32 and the
// half l / 32 of the kz spectrum (h in [half KZH / 2, (half + 1) KZH / 2)), so each lane holds
// half of a column's coefficients and the two halves' partial sums meet in one lane swap.  Wave
// w handles the z planes w, w + 8, ... of the block's columns.  The block's z twiddles
// exp(+2 pi i h z / pz) are staged in LDS (tz[z][h], KZH per row) and read as broadcasts, each
// shared by the three fields a block contracts.

// this lane's half of the column of one field (h < kzh; zero past kzh).  Every load is made,
// at the clamped plane past kzh, and zeroed afterwards: a guarded load compiles to a branch and
// a wait per load, an unguarded one lets all of them be in flight together.
template <int KZH>
__device__ __forceinline__ void load_half(const float2* __restrict__ Fc, size_t hstride, int kzh,
                                          int half, float2* F) {
  constexpr int NHH = KZH / 2;
  float2 v[NHH];
#pragma unroll
  for (int u = 0; u < NHH; ++u) v[u] = Fc[(size_t)min(half * NHH + u, kzh - 1) * hstride];
#pragma unroll
  for (int u = 0; u < NHH; ++u) F[u] = half * NHH + u < kzh ? v[u] : make_float2(0.f, 0.f);
}

// the block's z twiddles tz[z][h] (zero past kzh): pz * KZH <= 48 * 16 entries, two per thread;
// the loads are issued here and the LDS stores made later by tz_store, so that the caller's
// other loads are in flight at the same time
template <int KZH>
struct TzStage {
  Stager<64 * kColWaves, 2> st;
  __device__ __forceinline__ void load(const float2* __restrict__ tw_zT, int pz, int kzh) {
    st.load(pz * KZH, 0, [&](int o) {
      const int z = o / KZH, h = o - z * KZH;
      return tw_zT[(size_t)z * kZP + min(h, kzh - 1)];
    });
  }
  __device__ __forceinline__ void store(int pz, int kzh, float2* tz) const {
    st.store(pz * KZH, 0, [&](int o, float2 v) {
      const int h = o % KZH;
      tz[o] = h < kzh ? v : make_float2(0.f, 0.f);
    });
  }
};

// f_j(z) = Re F_j[0] + 2 sum_{h >= 1} Re(F_j[h] tz[z][h]) for three fields at one plane z: each
// half sums its h range, then the halves exchange partial sums (lane l <-> l ^ 32)
template <int KZH>
__device__ __forceinline__ void iota_z3(const float2 (*F)[KZH / 2], const float2* tz, int z,
                                        int half, float* f) {
  constexpr int NHH = KZH / 2;
#pragma unroll
  for (int j = 0; j < 3; ++j) f[j] = 0.f;
#pragma unroll
  for (int u = 0; u < NHH; ++u) {
    const int h = half * NHH + u;
    const float2 t = tz[z * KZH + h];
    const float sc = h == 0 ? 1.f : 2.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      f[j] = fmaf(sc * F[j][u].x, t.x, f[j]);
      f[j] = fmaf(-sc * F[j][u].y, t.y, f[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) f[j] += __shfl_xor(f[j], 32);
}

// Forward stage, block (column chunk, component i): f_(i,j)(z) = iota_z(F2[i dim + j]);
// out(z) = sum_j f_(i,j)(z) V_j(z) (+ sum_j DUGr_(i,j)(z) DVP_j(z) for products); the state
// pass stores DUGw_(i,j)(z) = f_(i,j)(z); G[i][h] = sum_z out(z) conj tz[z][h], wave w taking
// h = half KZH / 2 + w.
template <int NZS, int KZH, bool INC>
__global__ __launch_bounds__(64 * kColWaves) void k_fx_col_fwd(Geo gp, const float2* __restrict__ F2,
                                                    const float* __restrict__ VP,
                                                    float* __restrict__ DUGw,
                                                    const float* __restrict__ DUGr,
                                                    const float* __restrict__ DVP,
                                                    const float2* __restrict__ tw_zT,
                                                    float2* __restrict__ G) {
  __shared__ float2 tz[kColWaves * NZS * KZH];
  __shared__ float buf[kColWaves * NZS][kColW];
  const int lane = threadIdx.x & 63;
  const int col = lane & (kColW - 1), half = lane >> 5;
  const int w = wave_uniform(threadIdx.x >> 6);
  const int i = blockIdx.y;
  const int nq = gp.nx * gp.ny;
  const int q = blockIdx.x * kColW + col;
  const int qc = q < nq ? q : nq - 1;
  const bool live = q < nq;
  const int pz = gp.nz, kzh = gp.kzh;
  const int64_t MP = gp.M;
  float2 F[3][KZH / 2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    load_half<KZH>(F2 + (size_t)(3 * i + j) * kzh * nq + qc, (size_t)nq, kzh, half, F[j]);
  TzStage<KZH> tzs;
  tzs.load(tw_zT, pz, kzh);
  // planes past pz are computed at the clamped plane pz - 1 and not stored: no branch keeps the
  // loads of later planes from being issued early.  Every load of the block's inputs is issued
  // before the first LDS store and barrier.
  float vp[3][NZS], dg[3][NZS], dw[3][NZS];
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int64_t at = (int64_t)min(w + kColWaves * s, pz - 1) * nq + qc;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      vp[j][s] = VP[j * MP + at];
      if (INC) {
        dg[j][s] = DUGr[(int64_t)(3 * i + j) * MP + at];
        dw[j][s] = DVP[j * MP + at];
      }
    }
  }
  tzs.store(pz, kzh, tz);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int z = w + kColWaves * s;
    const int zc = min(z, pz - 1);
    const int64_t at = (int64_t)zc * nq + qc;
    float f[3];
    iota_z3<KZH>(F, tz, zc, half, f);
    float o = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o = fmaf(f[j], vp[j][s], o);
      const int64_t ac = (int64_t)(3 * i + j) * MP + at;
      if (INC) o = fmaf(dg[j][s], dw[j][s], o);
      else if (live && half == 0 && z < pz) DUGw[ac] = f[j];
    }
    if (half == 0) buf[z][col] = o;
  }
  __syncthreads();
  if (!live) return;
  const int h = half * (KZH / 2) + w;
  if (w >= KZH / 2 || h >= kzh) return;
  float2 a = make_float2(0.f, 0.f), b = a;
  int z = 0;
#pragma unroll 4
  for (; z + 1 < pz; z += 2) {
    const float v0 = buf[z][col], v1 = buf[z + 1][col];
    const float2 t0 = tz[z * KZH + h], t1 = tz[(z + 1) * KZH + h];
    a.x = fmaf(v0, t0.x, a.x);
    a.y = fmaf(-v0, t0.y, a.y);
    b.x = fmaf(v1, t1.x, b.x);
    b.y = fmaf(-v1, t1.y, b.y);
  }
  if (z < pz) {
    const float v0 = buf[z][col];
    const float2 t0 = tz[z * KZH + h];
    a.x = fmaf(v0, t0.x, a.x);
    a.y = fmaf(-v0, t0.y, a.y);
  }
  G[((size_t)i * kzh + h) * nq + q] = make_float2(a.x + b.x, a.y + b.y);
}

// Backward stage, block (column chunk, component j): kg_i(z) = iota_z(F2[i]) of the cotangent;
// GACC_j (+)= sum_i DUG_(i,j)(z) kg_i(z); G[i dim + j][h] = sum_z kg_i(z) V_j(z) conj tz[z][h]
// for i < 3, wave w taking h = half KZH / 2 + w.
template <int NZS, int KZH, bool UNUSED>
__global__ __launch_bounds__(64 * kColWaves) void k_fx_col_bwd(Geo gp, const float2* __restrict__ F2,
                                                    const float* __restrict__ VP,
                                                    const float* __restrict__ DUG,
                                                    float* __restrict__ GACC, int first,
                                                    const float2* __restrict__ tw_zT,
                                                    float2* __restrict__ G) {
  __shared__ float2 tz[kColWaves * NZS * KZH];
  __shared__ float bk[3][kColWaves * NZS][kColW];   // kg_i(z) V_j(z)
  const int lane = threadIdx.x & 63;
  const int col = lane & (kColW - 1), half = lane >> 5;
  const int w = wave_uniform(threadIdx.x >> 6);
  const int j = blockIdx.y;
  const int nq = gp.nx * gp.ny;
  const int q = blockIdx.x * kColW + col;
  const int qc = q < nq ? q : nq - 1;
  const bool live = q < nq;
  const int pz = gp.nz, kzh = gp.kzh;
  const int64_t MP = gp.M;
  float2 F[3][KZH / 2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    load_half<KZH>(F2 + (size_t)c * kzh * nq + qc, (size_t)nq, kzh, half, F[c]);
  TzStage<KZH> tzs;
  tzs.load(tw_zT, pz, kzh);
  // the planes' accumulator, state derivatives and velocity, loaded before the barrier
  float ga[NZS], du[3][NZS], vv[NZS];
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int64_t at = (int64_t)min(w + kColWaves * s, pz - 1) * nq + qc;
    ga[s] = GACC[j * MP + at];
    vv[s] = VP[j * MP + at];
#pragma unroll
    for (int c = 0; c < 3; ++c) du[c][s] = DUG[(int64_t)(3 * c + j) * MP + at];
  }
  tzs.store(pz, kzh, tz);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int z = w + kColWaves * s;
    const int64_t at = (int64_t)min(z, pz - 1) * nq + qc;
    float kg[3];
    iota_z3<KZH>(F, tz, min(z, pz - 1), half, kg);
    float a = first ? 0.f : ga[s];
#pragma unroll
    for (int c = 0; c < 3; ++c) a = fmaf(du[c][s], kg[c], a);
    if (live && half == 0 && z < pz) GACC[j * MP + at] = a;
    const float vj = vv[s];
    if (half == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) bk[c][z][col] = kg[c] * vj;
    }
  }
  __syncthreads();
  if (!live) return;
  const int h = half * (KZH / 2) + w;
  if (w >= KZH / 2 || h >= kzh) return;
  float2 a[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) a[c] = make_float2(0.f, 0.f);
#pragma unroll 4
  for (int z = 0; z < pz; ++z) {
    const float2 t = tz[z * KZH + h];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = bk[c][z][col];
      a[c].x = fmaf(v, t.x, a[c].x);
      a[c].y = fmaf(-v, t.y, a[c].y);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) G[((size_t)(3 * c + j) * kzh + h) * nq + q] = a[c];
}

// ------------------------------------------------------------------------------ 3. pi yx
// LDS layout of a yx block: the G plane, the x-stage result, R, and the block's twiddles
struct YxLds {
  float2 *Pl, *T, *Rs, *Tx, *Ty;
};
__device__ __forceinline__ YxLds yx_lds(const Geo& g, const Geo& gp, float2* base) {
  YxLds L;
  L.Pl = base;                                // [PY][PX + 1] (padded rows)
  L.T = L.Pl + (size_t)gp.ny * (gp.nx + 1);   // [PY][kKC]
  L.Rs = L.T + (size_t)gp.ny * kKC;           // [KY][kKC]
  L.Tx = L.Rs + (size_t)g.ky * kKC;           // [PX][kKC]: Tx[jx][x] of the block's kx chunk
  L.Ty = L.Tx + (size_t)gp.nx * kKC;          // [PY][KY]
  return L;
}
// the block's twiddles into LDS (once per block); one round of loads in flight together up to
// 64 x values and 48 x 32 (y, ky) pairs
__device__ __forceinline__ void yx_twiddles(const Geo& g, const Geo& gp,
                                            const float2* __restrict__ tw_xT,
                                            const float2* __restrict__ tw_yT, int kyp, int k0,
                                            const YxLds& L) {
  const int KX = g.kx, KY = g.ky, PX = gp.nx, PY = gp.ny;
  const int nX = PX * kKC, nY = PY * KY;
  const int rounds = max((nX + 255) / 256, (nY + 1535) / 1536);
  for (int r = 0; r < rounds; ++r) {
    Stager<256, 1> sx;
    Stager<256, 6> sy;
    sx.load(nX, r * 256, [&](int o) {
      const int x = o / kKC, kl = o - x * kKC;
      return tw_xT[(size_t)x * KX + min(k0 + kl, KX - 1)];
    });
    sy.load(nY, r * 1536, [&](int o) {
      const int y = o / KY, jy = o - y * KY;
      return tw_yT[(size_t)y * kyp + jy];
    });
    sx.store(nX, r * 256, [&](int o, float2 v) { L.Tx[o] = v; });
    sy.store(nY, r * 1536, [&](int o, float2 v) { L.Ty[o] = v; });
  }
}

// R[jy][kl] = sum_y sum_x G[y][x] conj Tx[jx][x] conj Ty[jy][y] for the block's kx chunk, the
// G plane (c, h) staged in LDS; R for (jy, jx = k0 + kl) lands in L.Rs.  Starts and ends with a
// block barrier.
__device__ __forceinline__ void pi_yx_passes(const Geo& g, const Geo& gp, const YxLds& L);

// a G plane held in registers, kPlaneRegs entries per thread (entry o = threadIdx.x + 256 u)
constexpr int kPlaneRegs = 24;
__device__ __forceinline__ void plane_to_regs(const float2* __restrict__ Gp, int n, float2* R) {
#pragma unroll
  for (int u = 0; u < kPlaneRegs; ++u) {
    const int o = threadIdx.x + 256 * u;
    R[u] = o < n ? Gp[o] : make_float2(0.f, 0.f);
  }
}
__device__ __forceinline__ void regs_to_lds(const float2* R, int PX, int n, float2* Pl) {
#pragma unroll
  for (int u = 0; u < kPlaneRegs; ++u) {
    const int o = threadIdx.x + 256 * u;
    if (o < n) {
      const int y = o / PX;
      Pl[y * (PX + 1) + (o - y * PX)] = R[u];
    }
  }
}

// the x and y contractions of the plane staged in L.Pl (a block barrier first and last)
__device__ __forceinline__ void pi_yx_passes(const Geo& g, const Geo& gp, const YxLds& L) {
  const int KY = g.ky, PX = gp.nx, PY = gp.ny, SP = PX + 1;
  __syncthreads();
  for (int o = threadIdx.x; o < PY * kKC; o += 256) {
    const int y = o / kKC, kl = o - y * kKC;
    float2 a = make_float2(0.f, 0.f), b = a;
    int x = 0;
#pragma unroll 4
    for (; x + 1 < PX; x += 2) {
      cmac_conj(a, L.Pl[y * SP + x], L.Tx[x * kKC + kl]);
      cmac_conj(b, L.Pl[y * SP + x + 1], L.Tx[(x + 1) * kKC + kl]);
    }
    if (x < PX) cmac_conj(a, L.Pl[y * SP + x], L.Tx[x * kKC + kl]);
    L.T[o] = make_float2(a.x + b.x, a.y + b.y);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < KY * kKC; o += 256) {
    const int jy = o / kKC, kl = o - jy * kKC;
    float2 a = make_float2(0.f, 0.f), b = a;
    int y = 0;
#pragma unroll 4
    for (; y + 1 < PY; y += 2) {
      cmac_conj(a, L.T[y * kKC + kl], L.Ty[y * KY + jy]);
      cmac_conj(b, L.T[(y + 1) * kKC + kl], L.Ty[(y + 1) * KY + jy]);
    }
    if (y < PY) cmac_conj(a, L.T[y * kKC + kl], L.Ty[y * KY + jy]);
    L.Rs[o] = make_float2(a.x + b.x, a.y + b.y);
  }
  __syncthreads();
}

// the band entries a thread of a yx block writes: entry k = (jx, jy, kz0 + h) with value R and,
// where its mirror is written by the same thread, the mirror -k with conj(R).  Unpaired entries
// (jx = 0 or jy = 0) are written as zero by their own k; the unpaired plane jz = 0 by h = 0.
struct Target {
  int b;        // band index of k
  int bm;       // band index of -k, or -1
  int bz;       // unpaired k with h > 0: the unpaired entry (jx, jy) of the plane kz = -h, else -1
  bool zero;    // k is unpaired
  bool real;    // k = 0
};

__device__ __forceinline__ Target target(const Geo& g, int h, int jx, int jy) {
  Target t;
  const int jz = g.kz0 + h;
  t.b = (jz * g.ky + jy) * g.kx + jx;
  t.zero = jx == 0 || jy == 0;
  t.real = false;
  t.bm = -1;
  t.bz = -1;
  if (t.zero) {
    if (h > 0) t.bz = ((g.kz0 - h) * g.ky + jy) * g.kx + jx;
    return t;
  }
  const int mx = g.kx - jx, my = g.ky - jy;
  if (h > 0) {
    t.bm = ((g.kz0 - h) * g.ky + my) * g.kx + mx;
  } else {
    const int ky = jy - g.ky / 2, kx = jx - g.kx / 2;
    const bool own = ky > 0 || (ky == 0 && kx >= 0);
    if (!own) {
      t.b = -1;   // written by the owner of -k
      return t;
    }
    if (ky == 0 && kx == 0) t.real = true;
    else t.bm = (g.kz0 * g.ky + my) * g.kx + mx;
  }
  return t;
}

// the band values a forward stage update of component i at band index b reads (b < 0: a
// harmless in-bounds load of entry 0, not used)
struct StageIn {
  float2 s, u, p;
};
__device__ __forceinline__ StageIn stage_load(const Geo& g, int i, int b,
                                              const float2* __restrict__ src,
                                              const float2* __restrict__ un,
                                              const float2* __restrict__ acc) {
  const size_t o = (size_t)i * g.B + max(b, 0);
  return StageIn{src[o], un[o], acc[o]};
}

// Forward stage update of component i at band index b with conv (unscaled)
__device__ __forceinline__ void stage_entry(const Geo& g, int i, int b, float2 cv, float scaleP,
                                            const StageIn& in, float2* __restrict__ acc, int st,
                                            float2* __restrict__ wout) {
  const size_t o = (size_t)i * g.B + b;
  const float h = g.dt;
  const float2 sv = in.s;
  const float2 k = make_float2(-sv.x - scaleP * cv.x, -sv.y - scaleP * cv.y);
  const float2 u = in.u;
  float2 a;
  if (st == 1) {
    a = k;
  } else {
    const float2 p = in.p;
    const float f = st == 4 ? 1.f : 2.f;
    a = make_float2(fmaf(f, k.x, p.x), fmaf(f, k.y, p.y));
  }
  if (st < 4) {
    acc[o] = a;
    const float c = st == 3 ? h : 0.5f * h;
    wout[o] = make_float2(fmaf(c, k.x, u.x), fmaf(c, k.y, u.y));
  } else {
    const float s6 = h / 6.f;
    wout[o] = make_float2(fmaf(s6, a.x, u.x), fmaf(s6, a.y, u.y));
  }
}

__device__ __forceinline__ void stage_zero(const Geo& g, int i, int b, float2* __restrict__ acc,
                                           int st, float2* __restrict__ wout) {
  const size_t o = (size_t)i * g.B + b;
  if (st < 4) acc[o] = make_float2(0.f, 0.f);
  wout[o] = make_float2(0.f, 0.f);
}

// block (i * kzh + h, kx chunk); NO = output entries (jy, kl) per thread.  The G plane, the
// twiddles and the band values of the thread's entries are all loaded before the first barrier.
template <int NO>
__global__ __launch_bounds__(256) void k_fx_pi_yx_stage(Geo g, Geo gp, const float2* __restrict__ G,
                                                        const float2* __restrict__ tw_xT,
                                                        const float2* __restrict__ tw_yT, int kyp,
                                                        float scaleP,
                                                        const float2* __restrict__ src,
                                                        const float2* __restrict__ un,
                                                        float2* __restrict__ acc, int st,
                                                        float2* __restrict__ wout) {
  extern __shared__ float2 lds[];
  const int KY = g.ky, PX = gp.nx, PY = gp.ny;
  const YxLds L = yx_lds(g, gp, lds);
  const float2* Rs = L.Rs;
  const int ih = blockIdx.x;
  const int i = ih / g.kzh, h = ih - i * g.kzh;
  const int k0 = blockIdx.y * kKC;
  const int np = PY * PX;
  float2 R[kPlaneRegs];
  plane_to_regs(G + (size_t)ih * np, np, R);
  Target t[NO];
  StageIn in[NO][2];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int o = threadIdx.x + 256 * u;
    const int jy = o / kKC, kl = o - jy * kKC;
    const int jx = k0 + kl;
    t[u] = target(g, h, min(jx, g.kx - 1), min(jy, KY - 1));
    if (o >= KY * kKC || jx >= g.kx) t[u].b = -1;   // no entry for this slot
    in[u][0] = stage_load(g, i, t[u].zero ? -1 : t[u].b, src, un, acc);
    in[u][1] = stage_load(g, i, t[u].bm, src, un, acc);
  }
  yx_twiddles(g, gp, tw_xT, tw_yT, kyp, k0, L);
  regs_to_lds(R, PX, np, L.Pl);
  pi_yx_passes(g, gp, L);
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int o = threadIdx.x + 256 * u;
    const Target& tu = t[u];
    if (tu.b < 0) continue;
    if (tu.zero) {
      stage_zero(g, i, tu.b, acc, st, wout);
      if (tu.bz >= 0) stage_zero(g, i, tu.bz, acc, st, wout);
      continue;
    }
    float2 r = Rs[o];
    if (tu.real) r.y = 0.f;
    stage_entry(g, i, tu.b, r, scaleP, in[u][0], acc, st, wout);
    if (tu.bm >= 0) stage_entry(g, i, tu.bm, make_float2(r.x, -r.y), scaleP, in[u][1], acc, st, wout);
  }
  if (h == 0 && blockIdx.y == 0) {   // the unpaired plane kz = -K/2
    for (int o = threadIdx.x; o < g.ky * g.kx; o += 256) stage_zero(g, i, o, acc, st, wout);
  }
}

// the band values a transposed-sweep update of component i at band index b reads (b < 0: a
// harmless in-bounds load of entry 0, not used)
struct AdjIn {
  float2 r, p, ks;
};
__device__ __forceinline__ AdjIn adj_load(const Geo& g, int i, int b,
                                          const float2* __restrict__ rho,
                                          const float2* __restrict__ Asum,
                                          const float2* __restrict__ Ksum) {
  const size_t o = (size_t)i * g.B + max(b, 0);
  return AdjIn{rho[o], Asum[o], Ksum[o]};
}

// Transposed-sweep update of component i at band index b with A = sum_j i q_j R_j / MP
__device__ __forceinline__ void adj_entry(const Geo& g, int i, int b, float2 A, int st, int more,
                                          const AdjIn& in, float2* __restrict__ rho,
                                          float2* __restrict__ Asum, float2* __restrict__ Ksum,
                                          float2* __restrict__ kap) {
  const size_t o = (size_t)i * g.B + b;
  const float h = g.dt;
  const float cr = st == 2 ? h / 6.f : h / 3.f;
  const float ca = st == 4 ? h : 0.5f * h;
  const float2 r = in.r;
  float2 as = A;
  if (st != 4) {
    const float2 p = in.p;
    as = make_float2(p.x + A.x, p.y + A.y);
  }
  float2 kp;
  if (st > 1) {
    Asum[o] = as;
    kp = make_float2(fmaf(ca, A.x, cr * r.x), fmaf(ca, A.y, cr * r.y));
  } else {
    const float2 rn = make_float2(r.x + as.x, r.y + as.y);
    rho[o] = rn;
    if (!more) return;
    kp = make_float2(h / 6.f * rn.x, h / 6.f * rn.y);
  }
  kap[o] = kp;
  const float2 ks = in.ks;
  Ksum[o] = make_float2(ks.x + kp.x, ks.y + kp.y);
}

// Transposed-sweep yx block (i * kzh + h, kx chunk); NO = output entries (jy, kl) per thread.
// A = i scaleP sum_j q_j R_j with R_j = Y(X(G_j)) and q_j the derivative symbol of axis j.  q_x
// depends on kx only and q_z is constant in the block, so both commute with the y contraction:
//   A = i scaleP [Y(q_x X(G_0) + q_z X(G_2)) + q_y Y(X(G_1))].
// The three G planes are staged in LDS together; one x pass forms T02 = q_x X(G_0) + q_z X(G_2)
// and T1 = X(G_1), one y pass both y sums.  All global loads (planes, twiddles, the band entries
// the thread updates) are issued before the first barrier.
constexpr int kAdjRegs = 9;   // plane entries per thread and round (one round for 48 x 48)

__host__ __device__ __forceinline__ size_t adj_plane_stride(const Geo& gp) {
  return (size_t)gp.ny * (gp.nx + 1);
}

template <int NO>
__global__ __launch_bounds__(256) void k_fx_pi_yx_adj(Geo g, Geo gp, const float2* __restrict__ G,
                                                      const float2* __restrict__ tw_xT,
                                                      const float2* __restrict__ tw_yT, int kyp,
                                                      float scaleP, float2* __restrict__ rho,
                                                      float2* __restrict__ Asum,
                                                      float2* __restrict__ Ksum,
                                                      float2* __restrict__ kap, int st, int more) {
  extern __shared__ float2 lds[];
  const int KX = g.kx, KY = g.ky, PX = gp.nx, PY = gp.ny, SP = PX + 1;
  const size_t PS = adj_plane_stride(gp);
  float2* Pl = lds;                      // [3][PY][SP]
  float2* T02 = Pl + 3 * PS;             // [PY][kKC]
  float2* T1 = T02 + (size_t)PY * kKC;   // [PY][kKC]
  float2* Tx = T1 + (size_t)PY * kKC;    // [PX][kKC]
  float2* Ty = Tx + (size_t)PX * kKC;    // [PY][KY]
  const int ih = blockIdx.x;
  const int i = ih / g.kzh, h = ih - i * g.kzh;
  const int k0 = blockIdx.y * kKC;
  const int jz = g.kz0 + h;
  const int np = PY * PX;
  const float2* Gp[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) Gp[j] = G + ((size_t)(3 * i + j) * g.kzh + h) * np;
  // the band entries this thread updates, loaded first
  Target t[NO];
  AdjIn in[NO][3];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int o = threadIdx.x + 256 * u;
    const int jy = o / kKC, kl = o - jy * kKC;
    const int jx = k0 + kl;
    t[u] = target(g, h, min(jx, KX - 1), min(jy, KY - 1));
    if (o >= KY * kKC || jx >= KX) t[u].b = -1;   // no entry for this slot
    in[u][0] = adj_load(g, i, t[u].b, rho, Asum, Ksum);
    in[u][1] = adj_load(g, i, t[u].bm, rho, Asum, Ksum);
    in[u][2] = adj_load(g, i, t[u].bz, rho, Asum, Ksum);
  }
  // the three planes, kAdjRegs entries of each per thread and round, then the twiddles
  const int rounds = (np + 256 * kAdjRegs - 1) / (256 * kAdjRegs);
  for (int r = 0; r < rounds; ++r) {
    const int base = r * 256 * kAdjRegs;
    Stager<256, kAdjRegs> sp[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) sp[j].load(np, base, [&](int o) { return Gp[j][o]; });
    if (r == 0) yx_twiddles(g, gp, tw_xT, tw_yT, kyp, k0, YxLds{nullptr, nullptr, nullptr, Tx, Ty});
#pragma unroll
    for (int j = 0; j < 3; ++j)
      sp[j].store(np, base, [&](int o, float2 v) {
        const int y = o / PX;
        Pl[j * PS + y * SP + (o - y * PX)] = v;
      });
  }
  __syncthreads();
  // x pass: (y, kl) outputs, the three planes' sums together
  const float qz = qaxis(g, 2, jz);
  for (int o = threadIdx.x; o < PY * kKC; o += 256) {
    const int y = o / kKC, kl = o - y * kKC;
    const float qx = qaxis(g, 0, min(k0 + kl, KX - 1));
    float2 a0 = make_float2(0.f, 0.f), a1 = a0, a2 = a0;
    const float2* r0 = Pl + y * SP;
    const float2* r1 = r0 + PS;
    const float2* r2 = r1 + PS;
#pragma unroll 4
    for (int x = 0; x < PX; ++x) {
      const float2 tw = Tx[x * kKC + kl];
      cmac_conj(a0, r0[x], tw);
      cmac_conj(a1, r1[x], tw);
      cmac_conj(a2, r2[x], tw);
    }
    T02[o] = make_float2(fmaf(qx, a0.x, qz * a2.x), fmaf(qx, a0.y, qz * a2.y));
    T1[o] = a1;
  }
  __syncthreads();
  // y pass: A for the thread's outputs
  float2 A[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    A[u] = make_float2(0.f, 0.f);
    const int o = threadIdx.x + 256 * u;
    if (o >= KY * kKC) continue;
    const int jy = o / kKC, kl = o - jy * kKC;
    float2 s02 = make_float2(0.f, 0.f), s1 = s02;
#pragma unroll 4
    for (int y = 0; y < PY; ++y) {
      const float2 tw = Ty[y * KY + jy];
      cmac_conj(s02, T02[y * kKC + kl], tw);
      cmac_conj(s1, T1[y * kKC + kl], tw);
    }
    const float qy = qaxis(g, 1, jy);
    const float2 R = make_float2(fmaf(qy, s1.x, s02.x), fmaf(qy, s1.y, s02.y));
    A[u] = make_float2(-scaleP * R.y, scaleP * R.x);
  }
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const Target& tu = t[u];
    if (tu.b < 0) continue;
    float2 a = tu.zero ? make_float2(0.f, 0.f) : A[u];
    if (tu.real) a.y = 0.f;
    adj_entry(g, i, tu.b, a, st, more, in[u][0], rho, Asum, Ksum, kap);
    if (tu.bm >= 0)
      adj_entry(g, i, tu.bm, make_float2(a.x, -a.y), st, more, in[u][1], rho, Asum, Ksum, kap);
    if (tu.bz >= 0)
      adj_entry(g, i, tu.bz, make_float2(0.f, 0.f), st, more, in[u][2], rho, Asum, Ksum, kap);
  }
  if (h == 0 && blockIdx.y == 0) {   // the unpaired plane kz = -K/2: A = 0 there
    const int n = KY * KX;
    for (int base = 0; base < n; base += 1024) {
      AdjIn zin[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        zin[u] = adj_load(g, i, min(base + (int)threadIdx.x + 256 * u, n - 1), rho, Asum, Ksum);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = base + (int)threadIdx.x + 256 * u;
        if (o < n) adj_entry(g, i, o, make_float2(0.f, 0.f), st, more, zin[u], rho, Asum, Ksum, kap);
      }
    }
  }
}

int nzs_of(int pz) { return pz <= 16 ? 2 : pz <= 32 ? 4 : 6; }
int kzh_of(int kzh) { return kzh <= 8 ? 8 : 16; }

size_t lds_xy(const Geo& g, const Geo& gp) {
  return ((size_t)g.ky * (g.kx + 1) + (size_t)g.ky * kXC + (size_t)g.kx * kXC + (size_t)g.ky * gp.ny) *
         sizeof(float2);
}
size_t lds_yx_adj(const Geo& g, const Geo& gp) {
  return (3 * adj_plane_stride(gp) + 2 * (size_t)gp.ny * kKC + (size_t)gp.nx * kKC +
          (size_t)gp.ny * g.ky) *
         sizeof(float2);
}
size_t lds_yx(const Geo& g, const Geo& gp) {
  return ((size_t)gp.ny * (gp.nx + 1) + (size_t)gp.ny * kKC + (size_t)g.ky * kKC + (size_t)gp.nx * kKC +
          (size_t)gp.ny * g.ky) *
         sizeof(float2);
}

}  // namespace

bool fused_ok(const Geo& g, const Geo& gp) {
  return g.dim == 3 && gp.nz <= 48 && g.kzh <= 16 && g.kzh >= 2 && g.ky * kKC <= 4 * 256 &&
         gp.nx * gp.ny <= 256 * kPlaneRegs &&
         lds_xy(g, gp) <= 64 * 1024 && lds_yx(g, gp) <= 64 * 1024 &&
         lds_yx_adj(g, gp) <= 160 * 1024;
}

void fx_iota_xy(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* in, int deriv,
                float2* F2, hipStream_t s) {
  const int C = deriv ? g.dim * g.dim : g.dim;
  hipLaunchKernelGGL(k_fx_iota_xy, dim3(C * g.kzh, (gp.nx + kXC - 1) / kXC), dim3(256), lds_xy(g, gp),
                     s, g, gp, in, deriv, pl.tw_x, pl.tw_y, pl.nyp, F2);
}

#define COL_LAUNCH(KERNEL, NZS, KZH, ...)                                                 \
  do {                                                                                    \
    if (flag_)                                                                            \
      hipLaunchKernelGGL((KERNEL<NZS, KZH, true>), grid_, dim3(64 * kColWaves), 0, s,     \
                         __VA_ARGS__);                                                    \
    else                                                                                  \
      hipLaunchKernelGGL((KERNEL<NZS, KZH, false>), grid_, dim3(64 * kColWaves), 0, s,    \
                         __VA_ARGS__);                                                    \
  } while (0)
#define COL_KZH(KERNEL, NZS, ...)                                                         \
  do {                                                                                    \
    switch (kzh_of(gp.kzh)) {                                                             \
      case 8: COL_LAUNCH(KERNEL, NZS, 8, __VA_ARGS__); break;                             \
      default: COL_LAUNCH(KERNEL, NZS, 16, __VA_ARGS__); break;                           \
    }                                                                                     \
  } while (0)
#define NZS_DISPATCH(KERNEL, ...)                                                         \
  do {                                                                                    \
    const dim3 grid_((gp.nx * gp.ny + kColW - 1) / kColW, 3);                             \
    switch (nzs_of(gp.nz)) {                                                              \
      case 2: COL_KZH(KERNEL, 2, __VA_ARGS__); break;                                     \
      case 4: COL_KZH(KERNEL, 4, __VA_ARGS__); break;                                     \
      default: COL_KZH(KERNEL, 6, __VA_ARGS__); break;                                    \
    }                                                                                     \
  } while (0)

void fx_col_fwd(const Geo& gp, const DftPlan& pl, const float2* F2, const float* VP,
                float* DUGw, const float* DUGr, const float* DVP, float2* G, hipStream_t s) {
  const bool flag_ = DUGr != nullptr;   // products: read the stored stage derivatives
  NZS_DISPATCH(k_fx_col_fwd, gp, F2, VP, DUGw, DUGr, DVP, pl.tw_zT, G);
}

void fx_col_bwd(const Geo& gp, const DftPlan& pl, const float2* F2, const float* VP,
                const float* DUG, float* GACC, int first, float2* G, hipStream_t s) {
  const bool flag_ = false;
  NZS_DISPATCH(k_fx_col_bwd, gp, F2, VP, DUG, GACC, first, pl.tw_zT, G);
}

// output entries per thread of a yx block: ky * kKC <= 4 * 256 (fused_ok)
#define NO_DISPATCH(KERNEL, LDS, ...)                                                       \
  do {                                                                                      \
    const dim3 grid_(g.dim * g.kzh, (g.kx + kKC - 1) / kKC);                                \
    const size_t lds_ = (LDS);                                                              \
    switch ((g.ky * kKC + 255) / 256) {                                                     \
      case 1: hipLaunchKernelGGL(KERNEL<1>, grid_, dim3(256), lds_, s, __VA_ARGS__); break; \
      case 2: hipLaunchKernelGGL(KERNEL<2>, grid_, dim3(256), lds_, s, __VA_ARGS__); break; \
      case 3: hipLaunchKernelGGL(KERNEL<3>, grid_, dim3(256), lds_, s, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<4>, grid_, dim3(256), lds_, s, __VA_ARGS__); break; \
    }                                                                                       \
  } while (0)

void fx_pi_yx_stage(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                    const float2* src, const float2* un, float2* acc, int st, float2* wout,
                    hipStream_t s) {
  NO_DISPATCH(k_fx_pi_yx_stage, lds_yx(g, gp), g, gp, G, pl.tw_xT, pl.tw_yT, pl.kyp, scaleP,
              src, un, acc, st, wout);
}

void fx_pi_yx_adj(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                  float2* rho, float2* Asum, float2* Ksum, float2* kap, int st, int more,
                  hipStream_t s) {
  // the three staged planes take up to 160 KiB of LDS (fused_ok): allow the launches that size
  static std::once_flag once;
  std::call_once(once, [] {
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)k_fx_pi_yx_adj<1>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void*)k_fx_pi_yx_adj<2>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void*)k_fx_pi_yx_adj<3>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void*)k_fx_pi_yx_adj<4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipGetLastError();   // an attribute the runtime does not need leaves no error behind
  });
  NO_DISPATCH(k_fx_pi_yx_adj, lds_yx_adj(g, gp), g, gp, G, pl.tw_xT, pl.tw_yT, pl.kyp, scaleP,
              rho, Asum, Ksum, kap, st, more);
}

}  // namespace bl
