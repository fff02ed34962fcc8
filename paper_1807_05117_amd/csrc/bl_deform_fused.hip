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
//           plane and a chunk of kx, the G plane staged in LDS, followed by the band-side update
//           of the stage (forward) or of the transposed sweep (backward) at kz = h and at the
//           conjugate-mirror index -k.  On the kz = 0 plane the entry k is owned by the half
//           ky > 0 or (ky = 0, kx >= 0); its owner writes k and -k, so the result is exactly
//           Hermitian, and k = 0 takes the real part.
// Twiddle tables are those of the product grid's transform plan (bl_dft.hip layout).
#include "bl_internal.h"

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
  for (int o = threadIdx.x; o < KY * KX; o += 256) {
    const int jy = o / KX, jx = o - jy * KX;
    float2 v = plane[o];
    if (deriv) {
      const float q = cj == 0 ? qaxis(g, 0, jx) : (cj == 1 ? qaxis(g, 1, jy) : qaxis(g, 2, jz));
      v = make_float2(-q * v.y, q * v.x);
    }
    S[jy * SX + jx] = v;
  }
  for (int o = threadIdx.x; o < KX * kXC; o += 256) {
    const int jx = o / kXC, xl = o - jx * kXC;
    Txc[o] = tw_x[(size_t)jx * PX + min(x0 + xl, PX - 1)];
  }
  for (int o = threadIdx.x; o < KY * PY; o += 256) {
    const int jy = o / PY, y = o - jy * PY;
    Ty[o] = tw_y[(size_t)jy * nyp + y];
  }
  __syncthreads();
  // x: T[jy][xl] = sum_jx S[jy][jx] Tx[jx][x0 + xl]
  for (int o = threadIdx.x; o < KY * kXC; o += 256) {
    const int jy = o / kXC, xl = o - jy * kXC;
    float2 a = make_float2(0.f, 0.f), b = a;
    int jx = 0;
#pragma unroll 4
    for (; jx + 1 < KX; jx += 2) {
      cmac(a, S[jy * SX + jx], Txc[jx * kXC + xl]);
      cmac(b, S[jy * SX + jx + 1], Txc[(jx + 1) * kXC + xl]);
    }
    if (jx < KX) cmac(a, S[jy * SX + jx], Txc[jx * kXC + xl]);
    T[o] = make_float2(a.x + b.x, a.y + b.y);
  }
  __syncthreads();
  // y: F2[y][x0 + xl] = sum_jy T[jy][xl] Ty[jy][y]
  float2* dst = F2 + (size_t)ch * PY * PX;
  for (int o = threadIdx.x; o < PY * kXC; o += 256) {
    const int y = o / kXC, xl = o - y * kXC;
    if (x0 + xl >= PX) continue;
    float2 a = make_float2(0.f, 0.f), b = a;
    int jy = 0;
#pragma unroll 4
    for (; jy + 1 < KY; jy += 2) {
      cmac(a, T[jy * kXC + xl], Ty[jy * PY + y]);
      cmac(b, T[(jy + 1) * kXC + xl], Ty[(jy + 1) * PY + y]);
    }
    if (jy < KY) cmac(a, T[jy * kXC + xl], Ty[jy * PY + y]);
    dst[(size_t)y * PX + x0 + xl] = make_float2(a.x + b.x, a.y + b.y);
  }
}

// ---------------------------------------------------------------------------- 2. columns
// Block (32 columns, component), eight waves: lane l of a wave serves column l mod 32 and the
// half l / 32 of the kz spectrum (h in [half KZH / 2, (half + 1) KZH / 2)), so each lane holds
// half of a column's coefficients and the two halves' partial sums meet in one lane swap.  Wave
// w handles the z planes w, w + 8, ... of the block's columns.  The block's z twiddles
// exp(+2 pi i h z / pz) are staged in LDS (tz[z][h], KZH per row) and read as broadcasts, each
// shared by the three fields a block contracts.

// this lane's half of the column of one field (h < kzh; zero past kzh), loads issued together
template <int KZH>
__device__ __forceinline__ void load_half(const float2* __restrict__ Fc, size_t hstride, int kzh,
                                          int half, float2* F) {
  constexpr int NHH = KZH / 2;
#pragma unroll
  for (int u = 0; u < NHH; ++u) {
    const int h = half * NHH + u;
    F[u] = h < kzh ? Fc[(size_t)h * hstride] : make_float2(0.f, 0.f);
  }
}

template <int KZH>
__device__ __forceinline__ void stage_tz(const float2* __restrict__ tw_zT, int pz, int kzh,
                                         float2* tz) {
  for (int o = threadIdx.x; o < pz * KZH; o += 64 * kColWaves) {
    const int z = o / KZH, h = o - z * KZH;
    tz[o] = h < kzh ? tw_zT[(size_t)z * kZP + h] : make_float2(0.f, 0.f);
  }
}

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
  stage_tz<KZH>(tw_zT, pz, kzh, tz);
  // planes past pz are computed at the clamped plane pz - 1 and not stored: no branch keeps the
  // loads of later planes from being issued early
  float vp[3][NZS];
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int64_t at = (int64_t)min(w + kColWaves * s, pz - 1) * nq + qc;
#pragma unroll
    for (int j = 0; j < 3; ++j) vp[j][s] = VP[j * MP + at];
  }
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
      if (INC) o = fmaf(DUGr[ac], DVP[j * MP + at], o);
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
  stage_tz<KZH>(tw_zT, pz, kzh, tz);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NZS; ++s) {
    const int z = w + kColWaves * s;
    const int64_t at = (int64_t)min(z, pz - 1) * nq + qc;
    float kg[3];
    iota_z3<KZH>(F, tz, min(z, pz - 1), half, kg);
    const float g0 = GACC[j * MP + at];
    float a = first ? 0.f : g0;
#pragma unroll
    for (int c = 0; c < 3; ++c) a = fmaf(DUG[(int64_t)(3 * c + j) * MP + at], kg[c], a);
    if (live && half == 0 && z < pz) GACC[j * MP + at] = a;
    const float vj = VP[j * MP + at];
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
// the block's twiddles into LDS (once per block)
__device__ __forceinline__ void yx_twiddles(const Geo& g, const Geo& gp,
                                            const float2* __restrict__ tw_xT,
                                            const float2* __restrict__ tw_yT, int kyp, int k0,
                                            const YxLds& L) {
  const int KX = g.kx, KY = g.ky, PX = gp.nx, PY = gp.ny;
  for (int o = threadIdx.x; o < PX * kKC; o += 256) {
    const int x = o / kKC, kl = o - x * kKC;
    L.Tx[o] = tw_xT[(size_t)x * KX + min(k0 + kl, KX - 1)];
  }
  for (int o = threadIdx.x; o < PY * KY; o += 256) {
    const int y = o / KY, jy = o - y * KY;
    L.Ty[o] = tw_yT[(size_t)y * kyp + jy];
  }
}

// R[jy][kl] = sum_y sum_x G[y][x] conj Tx[jx][x] conj Ty[jy][y] for the block's kx chunk, the
// G plane (c, h) staged in LDS; R for (jy, jx = k0 + kl) lands in L.Rs.  Starts and ends with a
// block barrier.
__device__ __forceinline__ void pi_yx_passes(const Geo& g, const Geo& gp, const YxLds& L);

__device__ __forceinline__ void pi_yx_plane(const Geo& g, const Geo& gp,
                                            const float2* __restrict__ Gp, const YxLds& L) {
  const int PX = gp.nx, PY = gp.ny, SP = PX + 1;
  for (int o = threadIdx.x; o < PY * PX; o += 256) {
    const int y = o / PX;
    L.Pl[y * SP + (o - y * PX)] = Gp[o];
  }
  pi_yx_passes(g, gp, L);
}

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

// Forward stage update of component i at band index b with conv (unscaled)
__device__ __forceinline__ void stage_entry(const Geo& g, int i, int b, float2 cv, float scaleP,
                                            const float2* __restrict__ src,
                                            const float2* __restrict__ un,
                                            float2* __restrict__ acc, int st,
                                            float2* __restrict__ wout) {
  const size_t o = (size_t)i * g.B + b;
  const float h = g.dt;
  const float2 sv = src[o];
  const float2 k = make_float2(-sv.x - scaleP * cv.x, -sv.y - scaleP * cv.y);
  const float2 u = un[o];
  float2 a;
  if (st == 1) {
    a = k;
  } else {
    const float2 p = acc[o];
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

// block (i * kzh + h, kx chunk)
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
  yx_twiddles(g, gp, tw_xT, tw_yT, kyp, k0, L);
  pi_yx_plane(g, gp, G + (size_t)ih * PY * PX, L);
  for (int o = threadIdx.x; o < KY * kKC; o += 256) {
    const int jy = o / kKC, kl = o - jy * kKC;
    const int jx = k0 + kl;
    if (jx >= g.kx) continue;
    const Target t = target(g, h, jx, jy);
    if (t.b < 0) continue;
    if (t.zero) {
      stage_zero(g, i, t.b, acc, st, wout);
      if (t.bz >= 0) stage_zero(g, i, t.bz, acc, st, wout);
      continue;
    }
    float2 r = Rs[o];
    if (t.real) r.y = 0.f;
    stage_entry(g, i, t.b, r, scaleP, src, un, acc, st, wout);
    if (t.bm >= 0) stage_entry(g, i, t.bm, make_float2(r.x, -r.y), scaleP, src, un, acc, st, wout);
  }
  if (h == 0 && blockIdx.y == 0) {   // the unpaired plane kz = -K/2
    for (int o = threadIdx.x; o < g.ky * g.kx; o += 256) stage_zero(g, i, o, acc, st, wout);
  }
}

// Transposed-sweep update of component i at band index b with A = sum_j i q_j R_j / MP
__device__ __forceinline__ void adj_entry(const Geo& g, int i, int b, float2 A, int st, int more,
                                          float2* __restrict__ rho, float2* __restrict__ Asum,
                                          float2* __restrict__ Ksum, float2* __restrict__ kap) {
  const size_t o = (size_t)i * g.B + b;
  const float h = g.dt;
  const float cr = st == 2 ? h / 6.f : h / 3.f;
  const float ca = st == 4 ? h : 0.5f * h;
  const float2 r = rho[o];
  float2 as = A;
  if (st != 4) {
    const float2 p = Asum[o];
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
  const float2 ks = Ksum[o];
  Ksum[o] = make_float2(ks.x + kp.x, ks.y + kp.y);
}

__global__ __launch_bounds__(256) void k_fx_pi_yx_adj(Geo g, Geo gp, const float2* __restrict__ G,
                                                      const float2* __restrict__ tw_xT,
                                                      const float2* __restrict__ tw_yT, int kyp,
                                                      float scaleP, float2* __restrict__ rho,
                                                      float2* __restrict__ Asum,
                                                      float2* __restrict__ Ksum,
                                                      float2* __restrict__ kap, int st, int more) {
  extern __shared__ float2 lds[];
  const int KY = g.ky, PX = gp.nx, PY = gp.ny;
  const YxLds L = yx_lds(g, gp, lds);
  const float2* Rs = L.Rs;
  const int ih = blockIdx.x;
  const int i = ih / g.kzh, h = ih - i * g.kzh;
  const int k0 = blockIdx.y * kKC;
  const int jz = g.kz0 + h;
  yx_twiddles(g, gp, tw_xT, tw_yT, kyp, k0, L);
  // A for the thread's outputs, accumulated over j (at most 256 * 4 outputs per thread pass);
  // the next plane's loads are in flight while the current plane is contracted
  float2 A[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) A[u] = make_float2(0.f, 0.f);
  const int np = PY * PX;
  float2 R[kPlaneRegs];
  plane_to_regs(G + ((size_t)(3 * i) * g.kzh + h) * np, np, R);
  for (int j = 0; j < 3; ++j) {
    regs_to_lds(R, PX, np, L.Pl);
    if (j < 2) plane_to_regs(G + ((size_t)(3 * i + j + 1) * g.kzh + h) * np, np, R);
    pi_yx_passes(g, gp, L);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = threadIdx.x + 256 * u;
      if (o >= KY * kKC) break;
      const int jy = o / kKC, kl = o - jy * kKC;
      const int jx = min(k0 + kl, g.kx - 1);
      const float q = j == 0 ? qaxis(g, 0, jx) : (j == 1 ? qaxis(g, 1, jy) : qaxis(g, 2, jz));
      const float2 r = Rs[o];
      A[u].x = fmaf(-q * scaleP, r.y, A[u].x);
      A[u].y = fmaf(q * scaleP, r.x, A[u].y);
    }
    __syncthreads();   // Rs and Pl are rewritten by the next plane
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int o = threadIdx.x + 256 * u;
    if (o >= KY * kKC) break;
    const int jy = o / kKC, kl = o - jy * kKC;
    const int jx = k0 + kl;
    if (jx >= g.kx) continue;
    const Target t = target(g, h, jx, jy);
    if (t.b < 0) continue;
    float2 a = t.zero ? make_float2(0.f, 0.f) : A[u];
    if (t.real) a.y = 0.f;
    adj_entry(g, i, t.b, a, st, more, rho, Asum, Ksum, kap);
    if (t.bm >= 0) adj_entry(g, i, t.bm, make_float2(a.x, -a.y), st, more, rho, Asum, Ksum, kap);
    if (t.bz >= 0) adj_entry(g, i, t.bz, make_float2(0.f, 0.f), st, more, rho, Asum, Ksum, kap);
  }
  if (h == 0 && blockIdx.y == 0) {   // the unpaired plane kz = -K/2: A = 0 there
    for (int o = threadIdx.x; o < g.ky * g.kx; o += 256)
      adj_entry(g, i, o, make_float2(0.f, 0.f), st, more, rho, Asum, Ksum, kap);
  }
}

int nzs_of(int pz) { return pz <= 16 ? 2 : pz <= 32 ? 4 : 6; }
int kzh_of(int kzh) { return kzh <= 8 ? 8 : 16; }

size_t lds_xy(const Geo& g, const Geo& gp) {
  return ((size_t)g.ky * (g.kx + 1) + (size_t)g.ky * kXC + (size_t)g.kx * kXC + (size_t)g.ky * gp.ny) *
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
         lds_xy(g, gp) <= 64 * 1024 && lds_yx(g, gp) <= 64 * 1024;
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

void fx_pi_yx_stage(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                    const float2* src, const float2* un, float2* acc, int st, float2* wout,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_fx_pi_yx_stage, dim3(g.dim * g.kzh, (g.kx + kKC - 1) / kKC), dim3(256),
                     lds_yx(g, gp), s, g, gp, G, pl.tw_xT, pl.tw_yT, pl.kyp, scaleP, src, un, acc,
                     st, wout);
}

void fx_pi_yx_adj(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                  float2* rho, float2* Asum, float2* Ksum, float2* kap, int st, int more,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_fx_pi_yx_adj, dim3(g.dim * g.kzh, (g.kx + kKC - 1) / kKC), dim3(256),
                     lds_yx(g, gp), s, g, gp, G, pl.tw_xT, pl.tw_yT, pl.kyp, scaleP, rho, Asum,
                     Ksum, kap, st, more);
}

}  // namespace bl
