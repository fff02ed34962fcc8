// Mixed-precision z stages of the band <-> grid transforms (paper Section 3.1, iota and pi)
// on BF16 matrix cores with split operands and FP32 accumulation.
//
// Each z stage is a real matrix product over one axis:
//   iota:  v[z][q] = sum_j Wi[z][j] G[j][q],  G[2h] = Re F2[h], G[2h+1] = Im F2[h],
//          Wi[z][2h] = s_h cos(2 pi h z / nz), Wi[z][2h+1] = -s_h sin(2 pi h z / nz),
//          s_0 = 1, s_h = 2 (Hermitian half spectrum, real output)
//   pi:    G[j][q] = sum_z Wp[j][z] f[z][q],  Wp[2h][z] = cos(..), Wp[2h+1][z] = -sin(..)
// with q = (y, x) the column index.  Every FP32 operand x is split into two BF16 numbers,
// x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even), and each
// product is formed as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation; the dropped lo*lo term is below 2^-16 relative.  Twiddle splits are made on
// the host from FP64 values.
//
// Matrix-core operand layout (32x32x16, wave64): lane l holds A[i = l % 32][k = 8 (l / 32) + e]
// and B[k = 8 (l / 32) + e][j = l % 32] for e = 0..7; the accumulator register r of lane l
// holds D[i = 8 (r / 4) + 4 (l / 32) + r % 4][j = l % 32].
#include "bl_internal.h"

namespace bl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_to_f32(hi));
}

__device__ __forceinline__ f32x16 mfma3(bf16x8 ahi, bf16x8 alo, bf16x8 bhi, bf16x8 blo,
                                       f32x16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc, 0, 0, 0);
  return acc;
}

// iota z stage.  One wavefront per (component, 32 columns); the B operand (the half spectrum
// of its 32 columns) stays in registers while the wavefront walks all 32-plane z tiles.
// Wi is [2][nzp32][KP] BF16 (hi table then lo table), KP = 16 * KS.
template <int KS>
__global__ __launch_bounds__(256) void k_iota_z_mfma(Geo g, const float2* __restrict__ F2,
                                                     const unsigned short* __restrict__ Wi,
                                                     int nzp32, float* __restrict__ out,
                                                     int nqt) {
  BL_BATCH(g.bat)
  BL_AT(F2, g.bat);
  BL_AT(out, g.bat);
  constexpr int KP = 16 * KS;
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nq = g.nx * g.ny;
  const int c = blockIdx.y;
  if (wave >= nqt) return;
  const int q0 = wave * 32;
  const int col = lane & 31, kq = lane >> 5;
  const int q = q0 + col;
  const int qc = q < nq ? q : nq - 1;
  // B operand: k = 16 s + 8 kq + e  ->  h = 8 s + 4 kq + e/2, (Re, Im) by e parity
  bf16x8 bhi[KS], blo[KS];
  const float2* src = F2 + (size_t)c * g.kzh * nq + qc;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    u16x8 hv, lv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 8 * s + 4 * kq + i;
      const int hcl = h < g.kzh ? h : g.kzh - 1;
      float2 v = src[(size_t)hcl * nq];
      if (h >= g.kzh || q >= nq) v = make_float2(0.f, 0.f);
      unsigned short a, b;
      split_bf16(v.x, a, b);
      hv[2 * i] = a;
      lv[2 * i] = b;
      split_bf16(v.y, a, b);
      hv[2 * i + 1] = a;
      lv[2 * i + 1] = b;
    }
    bhi[s] = __builtin_bit_cast(bf16x8, hv);
    blo[s] = __builtin_bit_cast(bf16x8, lv);
  }
  const u16x8* Whi = reinterpret_cast<const u16x8*>(Wi);
  const u16x8* Wlo = reinterpret_cast<const u16x8*>(Wi + (size_t)nzp32 * KP);
  float* dst = out + (size_t)c * g.M + qc;
  // z tiles four at a time: the A operands of the four tiles are loaded before any product
  for (int zt0 = 0; zt0 * 32 < g.nz; zt0 += 4) {
    bf16x8 ahi[4][KS], alo[4][KS];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // A row of this lane; rows past the table (tiles beyond nz) reuse row 0, never stored
      const int zrow = (zt0 + u) * 32 < g.nz ? (zt0 + u) * 32 + col : col;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const size_t ai = ((size_t)zrow * KP + 16 * s + 8 * kq) / 8;
        ahi[u][s] = __builtin_bit_cast(bf16x8, Whi[ai]);
        alo[u][s] = __builtin_bit_cast(bf16x8, Wlo[ai]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int zt = zt0 + u;
      if (zt * 32 >= g.nz) break;
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s) acc = mfma3(ahi[u][s], alo[u][s], bhi[s], blo[s], acc);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int z = zt * 32 + 8 * (r >> 2) + 4 * kq + (r & 3);
        if (z < g.nz && q < nq) dst[(size_t)z * nq] = acc[r];
      }
    }
  }
}

// pi z stage.  One block of four wavefronts per (component, 32 columns); wavefront w takes
// the 16-plane steps w, w + 4, ... two at a time (16 loads in flight), splitting its B operand
// on the fly, for JT 32-row tiles of (Re, Im) outputs; the four partial accumulators are
// added in LDS in a fixed order.  Wp is [2][32 JT][nzp16] BF16 (hi table then lo table).
template <int JT>
__global__ __launch_bounds__(256) void k_pi_z_mfma(Geo g, const float* __restrict__ f,
                                                   const unsigned short* __restrict__ Wp,
                                                   int nzp16, float2* __restrict__ G) {
  BL_BATCH(g.bat)
  BL_AT(f, g.bat);
  BL_AT(G, g.bat);
  __shared__ float red[3][JT][16][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nq = g.nx * g.ny;
  const int c = blockIdx.y;
  const int q0 = blockIdx.x * 32;
  const int col = lane & 31, kq = lane >> 5;
  const int q = q0 + col;
  const int qc = q < nq ? q : nq - 1;
  f32x16 acc[JT];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  const float* src = f + (size_t)c * g.M + qc;
  const u16x8* Whi = reinterpret_cast<const u16x8*>(Wp);
  const u16x8* Wlo = reinterpret_cast<const u16x8*>(Wp + (size_t)32 * JT * nzp16);
  const int nsteps = (g.nz + 15) / 16;
  for (int s0 = w; s0 < nsteps; s0 += 8) {
    float v[2][8];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int z = 16 * (s0 + 4 * u) + 8 * kq + e;
        v[u][e] = src[(size_t)(z < g.nz ? z : g.nz - 1) * nq];
        if (z >= g.nz || q >= nq) v[u][e] = 0.f;
      }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int z0 = 16 * (s0 + 4 * u);
      if (z0 >= g.nz) break;
      u16x8 hv, lv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        unsigned short a, b;
        split_bf16(v[u][e], a, b);
        hv[e] = a;
        lv[e] = b;
      }
      const bf16x8 bhi = __builtin_bit_cast(bf16x8, hv);
      const bf16x8 blo = __builtin_bit_cast(bf16x8, lv);
#pragma unroll
      for (int t = 0; t < JT; ++t) {
        const size_t ai = ((size_t)(32 * t + col) * nzp16 + z0 + 8 * kq) / 8;
        acc[t] = mfma3(__builtin_bit_cast(bf16x8, Whi[ai]), __builtin_bit_cast(bf16x8, Wlo[ai]),
                       bhi, blo, acc[t]);
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) red[w - 1][t][r][lane] = acc[t][r];
  }
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      acc[t][r] = ((acc[t][r] + red[0][t][r][lane]) + red[1][t][r][lane]) + red[2][t][r][lane];
  // rows j = 8 (r / 4) + 4 kq + r % 4: registers (r, r + 1) with r % 4 in {0, 2} hold the
  // (Re, Im) pair of h = j / 2
  float2* dst = G + (size_t)c * g.kzh * nq + qc;
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int j = 32 * t + 8 * (r >> 2) + 4 * kq + (r & 3);
      const int h = j >> 1;
      if (h < g.kzh && q < nq) dst[(size_t)h * nq] = make_float2(acc[t][r], acc[t][r + 1]);
    }
}

}  // namespace

int mixed_kp(const Geo& g) { return (2 * g.kzh + 15) / 16 * 16; }
int mixed_jt(const Geo& g) { return (2 * g.kzh + 31) / 32; }

void iota_z_mixed(const Geo& g, const DftPlan& p, const float2* F2, int C, float* out,
                  hipStream_t s) {
  const int nq = g.nx * g.ny;
  const int nqt = (nq + 31) / 32;
  const dim3 grid = batch_grid(dim3((nqt + 3) / 4, C), g.bat);
  const int ks = mixed_kp(g) / 16;
#define L_IOTA(K)                                                                             \
  BL_LAUNCH(k_iota_z_mfma<K>, grid, dim3(256), 0, s, g, F2, p.wi_bf16, p.nzp32, out,          \
                     nqt)
  switch (ks) {
    case 1: L_IOTA(1); break;
    case 2: L_IOTA(2); break;
    case 3: L_IOTA(3); break;
    case 4: L_IOTA(4); break;
    case 5: L_IOTA(5); break;
    case 6: L_IOTA(6); break;
    case 7: L_IOTA(7); break;
    default: L_IOTA(8); break;
  }
#undef L_IOTA
}

void pi_z_mixed(const Geo& g, const DftPlan& p, const float* f, int C, float2* G, hipStream_t s) {
  const int nq = g.nx * g.ny;
  const dim3 grid = batch_grid(dim3((nq + 31) / 32, C), g.bat);
  switch (mixed_jt(g)) {
    case 1:
      BL_LAUNCH(k_pi_z_mfma<1>, grid, dim3(256), 0, s, g, f, p.wp_bf16, p.nzp16, G);
      break;
    case 2:
      BL_LAUNCH(k_pi_z_mfma<2>, grid, dim3(256), 0, s, g, f, p.wp_bf16, p.nzp16, G);
      break;
    case 3:
      BL_LAUNCH(k_pi_z_mfma<3>, grid, dim3(256), 0, s, g, f, p.wp_bf16, p.nzp16, G);
      break;
    default:
      BL_LAUNCH(k_pi_z_mfma<4>, grid, dim3(256), 0, s, g, f, p.wp_bf16, p.nzp16, G);
      break;
  }
}

}  // namespace bl
