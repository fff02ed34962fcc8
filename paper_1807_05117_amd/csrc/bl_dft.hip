// Band <-> grid transforms (paper Section 3.1, the inclusion iota and the projection pi) and
// the diagonal band operations (projected L~, spectral divergence, Hermitian projection).
//
//   iota(v~)(x_i) = Re sum_k v~(k) exp(2 pi i sum_j k_j i_j / n_j)
//   pi(f)(k)      = (1/M) sum_i f_i exp(-2 pi i sum_j k_j i_j / n_j)
//
// Both are separable truncated DFTs.  Admissible band vectors are Hermitian, so only the
// kz >= 0 half (kzh planes) is carried through the contractions:
//   iota:  x stage  F1[c][h][ky][x] = sum_kx v~[c][h][ky][kx] Tx[kx][x]
//          y stage  F2[c][h][y][x]  = sum_ky F1[c][h][ky][x] Ty[ky][y]
//          z stage  v[c][z][y][x]   = Re F2[c][0] + 2 sum_{h>=1} Re(F2[c][h] Tz[h][z])
//   pi:    z stage  G[c][h][y][x]   = sum_z f[c][z][y][x] conj Tz[h][z]
//          y stage  H[c][h][ky][x]  = sum_y G conj Ty[ky][y]
//          x stage  P[c][h][ky][kx] = sum_x H conj Tx[kx][x]
// and the kz < 0 half of pi is completed by Hermitian symmetry in band_finalize.
// The z stages touch every voxel and carry the bulk of the bytes; they keep one (y, x)
// column of the half spectrum in registers and stream the z planes, so every wavefront
// reads or writes whole contiguous rows.  Twiddles are FP32 values of exactly reduced
// angles computed on the host in FP64.
#include "bl_internal.h"

namespace bl {
namespace {

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

// ---------------------------------------------------------------------------- iota stages
// All contraction loops run in chunks of kU terms: the kU operand loads of a chunk are
// issued before its arithmetic, so kU memory latencies overlap.  Chunks past the end of an
// axis read clamped (in-bounds) data against zero-padded twiddle rows.

// x stage: one thread per (x, ky, c*kzh + h); the band row is uniform across the block.
__global__ __launch_bounds__(64) void k_iota_x(Geo g, const float2* __restrict__ band,
                                               const float2* __restrict__ tw_x,
                                               float2* __restrict__ F1) {
  BL_BATCH(g.bat)
  BL_AT(band, g.bat);
  BL_AT(F1, g.bat);
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int jy = blockIdx.y;
  const int ch = batch_bz(g.bat, bpair_);
  if (x >= g.nx) return;
  const int c = ch / g.kzh, h = ch - c * g.kzh;
  const float2* row = band + ((size_t)(c * g.kz + g.kz0 + h) * g.ky + jy) * g.kx;
  float2 a0 = make_float2(0.f, 0.f), a1 = a0;
  for (int j0 = 0; j0 < g.kx; j0 += kU) {
    float2 b[kU], t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      b[u] = row[min(j0 + u, g.kx - 1)];
      t[u] = tw_x[(size_t)(j0 + u) * g.nx + x];
    }
#pragma unroll
    for (int u = 0; u < kU; u += 2) {
      cmac(a0, b[u], t[u]);
      cmac(a1, b[u + 1], t[u + 1]);
    }
  }
  F1[((size_t)ch * g.ky + jy) * g.nx + x] = make_float2(a0.x + a1.x, a0.y + a1.y);
}

// y stage: one thread per (x, group of kYG y values, c*kzh + h); the F1 column is read once
// per group and the twiddles of the group are wave-uniform (scalar loads).
__global__ __launch_bounds__(64) void k_iota_y(Geo g, const float2* __restrict__ F1,
                                               const float2* __restrict__ tw_y, int nyp,
                                               float2* __restrict__ F2) {
  BL_BATCH(g.bat)
  BL_AT(F1, g.bat);
  BL_AT(F2, g.bat);
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y0 = blockIdx.y * kYG;
  const int ch = batch_bz(g.bat, bpair_);
  if (x >= g.nx) return;
  const float2* col = F1 + (size_t)ch * g.ky * g.nx + x;
  float2 acc[kYG];
#pragma unroll
  for (int u = 0; u < kYG; ++u) acc[u] = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < g.ky; j0 += kU) {
    float2 f[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) f[u] = col[(size_t)min(j0 + u, g.ky - 1) * g.nx];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float2* tw = tw_y + (size_t)(j0 + u) * nyp + y0;
#pragma unroll
      for (int v = 0; v < kYG; ++v) cmac(acc[v], f[u], tw[v]);
    }
  }
  float2* dst = F2 + ((size_t)ch * g.ny + y0) * g.nx + x;
#pragma unroll
  for (int u = 0; u < kYG; ++u)
    if (y0 + u < g.ny) dst[(size_t)u * g.nx] = acc[u];
}

// Fused x and y stages: one block per (c*kzh + h, tile of kFX columns, chunk of kFY rows).
// The band plane is staged in LDS (every lane of a wavefront reads the same entry), the x
// stage writes the block's columns of F1 for every ky to LDS, and the y stage forms the block's
// rows of F2 from them; F1 never goes through memory.  Each output is accumulated in exactly
// the order of k_iota_x / k_iota_y (two alternating partial sums over kx in chunks of kU; one
// sum over ky in chunks of kU, rows past ky against zero twiddle rows), so the results are
// bitwise those of the two separate stages.  A launch shape: the autotuner times it (16 or 32
// rows per block) against the two separate stages when the band plane and the block's F1
// tile fit kFusedLds bytes; every choice computes the same values.
constexpr int kFX = 64;
constexpr size_t kFusedLds = 64 * 1024;

template <int kFY>
__global__ __launch_bounds__(256) void k_iota_xy(Geo g, const float2* __restrict__ band,
                                                 const float2* __restrict__ tw_x,
                                                 const float2* __restrict__ tw_y, int nyp,
                                                 float2* __restrict__ F2) {
  BL_BATCH(g.bat)
  BL_AT(band, g.bat);
  BL_AT(F2, g.bat);
  extern __shared__ float2 lds_xy[];
  const int KX = g.kx, KY = g.ky;
  float2* S = lds_xy;                    // [KY][KX] band plane
  float2* T = S + (size_t)KY * KX;       // [KY][kFX] x-stage outputs of the block's columns
  const int ch = batch_bz(g.bat, bpair_);
  const int c = ch / g.kzh, h = ch - c * g.kzh;
  const float2* plane = band + (size_t)(c * g.kz + g.kz0 + h) * KY * KX;
  for (int i = threadIdx.x; i < KY * KX; i += 256) S[i] = plane[i];
  __syncthreads();
  const int xl = threadIdx.x & (kFX - 1);
  const int wq = wave_uniform(threadIdx.x >> 6);   // 4 wavefronts
  const int x = blockIdx.x * kFX + xl;
  const int xc = x < g.nx ? x : g.nx - 1;          // clamped column: loads stay in bounds
  // x stage: T[jy][xl] for jy = wq + 4 r, kNJ rows of a thread per pass sharing each twiddle
  // load (one round of kU loads per chunk for all of them)
  constexpr int kNJ = 8;
  for (int jb = wq; jb < KY; jb += 4 * kNJ) {
    float2 a0[kNJ], a1[kNJ];
#pragma unroll
    for (int r = 0; r < kNJ; ++r) a0[r] = a1[r] = make_float2(0.f, 0.f);
    for (int j0 = 0; j0 < KX; j0 += kU) {
      float2 t[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) t[u] = tw_x[(size_t)(j0 + u) * g.nx + xc];
#pragma unroll
      for (int r = 0; r < kNJ; ++r) {
        const float2* row = S + (size_t)min(jb + 4 * r, KY - 1) * KX;
#pragma unroll
        for (int u = 0; u < kU; u += 2) {
          cmac(a0[r], row[min(j0 + u, KX - 1)], t[u]);
          cmac(a1[r], row[min(j0 + u + 1, KX - 1)], t[u + 1]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kNJ; ++r) {
      const int jy = jb + 4 * r;
      if (jy < KY) T[jy * kFX + xl] = make_float2(a0[r].x + a1[r].x, a0[r].y + a1[r].y);
    }
  }
  __syncthreads();
  // y stage: rows y0 + wq + 4 v (v < kFY / 4) of the block's chunk, together per ky term
  constexpr int NV = kFY / 4;
  const int y0 = blockIdx.y * kFY + wq;
  float2 acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < KY; j0 += kU) {
    float2 f[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) f[u] = T[min(j0 + u, KY - 1) * kFX + xl];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float2* tw = tw_y + (size_t)(j0 + u) * nyp + y0;   // zero past ny and ky
#pragma unroll
      for (int v = 0; v < NV; ++v) cmac(acc[v], f[u], tw[4 * v]);
    }
  }
  if (x < g.nx) {
    float2* dst = F2 + (size_t)ch * g.ny * g.nx + x;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int y = y0 + 4 * v;
      if (y < g.ny) dst[(size_t)y * g.nx] = acc[v];
    }
  }
}

// z stage (real output): one thread per (column q, chunk of z, component); the half-spectrum
// column is held in registers.  Planes z and nz - z share their twiddles up to conjugation,
// so one pass over z <= nz/2 forms A = sum_h f.x t.x and B = sum_h f.y t.y and writes A - B
// to plane z and A + B to plane nz - z.  The block's twiddle rows are staged once in LDS;
// every lane of a wavefront reads the same entry (a broadcast), 16 bytes at a time.
template <int KZH>
__global__ __launch_bounds__(256) void k_iota_z(Geo g, const float2* __restrict__ F2,
                                                const float2* __restrict__ tw_zT,
                                                float* __restrict__ out, int zchunk) {
  BL_BATCH(g.bat)
  BL_AT(F2, g.bat);
  BL_AT(out, g.bat);
  extern __shared__ float4 tws4[];   // zchunk rows of KZH (even) or 2 (KZH == 1) float2
  constexpr int RW = KZH == 1 ? 2 : KZH;   // row width in float2
  float2* tws = reinterpret_cast<float2*>(tws4);
  const int nq = g.nx * g.ny;
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int c = batch_bz(g.bat, bpair_);
  const int zmax = g.nz / 2;
  const int z0 = blockIdx.y * zchunk;
  for (int i = threadIdx.x; i < zchunk * RW; i += 256) {
    const int r = i / RW, h = i - r * RW;
    tws[i] = h < KZH ? tw_zT[(size_t)min(z0 + r, zmax) * kZP + h] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  if (q >= nq) return;
  float2 f[RW];
  const float2* src = F2 + (size_t)c * g.kzh * nq + q;
#pragma unroll
  for (int h = 0; h < RW; ++h) {
    const int hc = h < g.kzh ? h : g.kzh - 1;   // clamped, always in bounds
    float2 v = src[(size_t)hc * nq];
    const float sc = h >= g.kzh ? 0.f : (h > 0 ? 2.f : 1.f);
    f[h] = make_float2(sc * v.x, sc * v.y);
  }
  const int z1 = min(zmax + 1, z0 + zchunk);
  float* dst = out + (size_t)c * g.M + q;
  for (int z = z0; z < z1; ++z) {
    const float4* t4 = tws4 + (size_t)(z - z0) * (RW / 2);
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int h2 = 0; h2 < RW / 2; ++h2) {
      const float4 t = t4[h2];
      a = fmaf(f[2 * h2].x, t.x, a);
      b = fmaf(f[2 * h2].y, t.y, b);
      a = fmaf(f[2 * h2 + 1].x, t.z, a);
      b = fmaf(f[2 * h2 + 1].y, t.w, b);
    }
    dst[(size_t)z * nq] = a - b;
    const int zm = g.nz - z;
    if (z > 0 && zm != z) dst[(size_t)zm * nq] = a + b;
  }
}

// ------------------------------------------------------------------------------ pi stages
// z stage: block of 64 columns x kNW wavefronts; in every round of kZU kNW planes wavefront
// w sums the planes w + u kNW (u < kZU) with wave-uniform twiddle rows -- kZU loads in
// flight per wavefront -- then the kNW partial sums are added in LDS in a fixed order.
constexpr int kNW = 8;
constexpr int kZU = 16;

template <int KZH>
// (up to 16 stored kz planes: at least 6 wavefronts per SIMD, i.e. three blocks of 8 per compute
// unit; unbounded, the compiler used 83 registers, two blocks fit and a 128^3 call took 15.3
// instead of 12.7 us)
__global__ __launch_bounds__(64 * kNW, KZH <= 16 ? 6 : 1) void k_pi_z(Geo g, const float* __restrict__ f,
                                                   const float2* __restrict__ tw_zT,
                                                   float2* __restrict__ G) {
  BL_BATCH(g.bat)
  BL_AT(f, g.bat);
  BL_AT(G, g.bat);
  constexpr int CH = (KZH % 8 == 0) ? 8 : ((KZH % 4 == 0) ? 4 : 1);
  __shared__ float2 sh[kNW - 1][CH][64];
  const int nq = g.nx * g.ny;
  const int tx = threadIdx.x;
  const int w = wave_uniform(threadIdx.y);
  const int q = blockIdx.x * 64 + tx;
  const int c = blockIdx.y;
  const int qc = q < nq ? q : nq - 1;   // clamped column: loads stay in bounds
  float2 acc[KZH];
#pragma unroll
  for (int h = 0; h < KZH; ++h) acc[h] = make_float2(0.f, 0.f);
  const float* src = f + (size_t)c * g.M + qc;
  for (int zb = 0; zb < g.nz; zb += kZU * kNW) {
    float v[kZU];
#pragma unroll
    for (int u = 0; u < kZU; ++u) v[u] = src[(size_t)min(zb + w + u * kNW, g.nz - 1) * nq];
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const float2* t = tw_zT + (size_t)(zb + w + u * kNW) * kZP;   // zero rows past nz
#pragma unroll
      for (int h = 0; h < KZH; ++h) {
        acc[h].x = fmaf(v[u], t[h].x, acc[h].x);
        acc[h].y = fmaf(-v[u], t[h].y, acc[h].y);
      }
    }
  }
#pragma unroll
  for (int h0 = 0; h0 < KZH; h0 += CH) {
    if (w > 0) {
#pragma unroll
      for (int hh = 0; hh < CH; ++hh) sh[w - 1][hh][tx] = acc[h0 + hh];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int hh = 0; hh < CH; ++hh) {
        float2 s = acc[h0 + hh];
#pragma unroll
        for (int o = 0; o < kNW - 1; ++o) {
          s.x += sh[o][hh][tx].x;
          s.y += sh[o][hh][tx].y;
        }
        acc[h0 + hh] = s;
      }
    }
    __syncthreads();
  }
  if (w == 0 && q < nq) {
    float2* dst = G + (size_t)c * g.kzh * nq + q;
#pragma unroll
    for (int h = 0; h < KZH; ++h)
      if (h < g.kzh) dst[(size_t)h * nq] = acc[h];
  }
}

// y stage: block of 64 x-columns x kYS wavefronts for one group of kJG ky outputs; wavefront
// s sums a contiguous 1/kYS of the y planes in chunks of kUY, the partial sums are added in
// LDS in a fixed order.
constexpr int kYS = 8;

__global__ __launch_bounds__(64 * kYS) void k_pi_y(Geo g, const float2* __restrict__ G,
                                                   const float2* __restrict__ tw_yT, int kyp,
                                                   int yseg, float2* __restrict__ H) {
  BL_BATCH(g.bat)
  BL_AT(G, g.bat);
  BL_AT(H, g.bat);
  __shared__ float2 sh[kYS - 1][kJG][64];
  const int tx = threadIdx.x;
  const int sgm = wave_uniform(threadIdx.y);
  const int x = blockIdx.x * 64 + tx;
  const int j0 = blockIdx.y * kJG;
  const int ch = batch_bz(g.bat, bpair_);
  const int xc = x < g.nx ? x : g.nx - 1;
  const float2* col = G + (size_t)ch * g.ny * g.nx + xc;
  float2 acc[kJG];
#pragma unroll
  for (int u = 0; u < kJG; ++u) acc[u] = make_float2(0.f, 0.f);
  const int ya = sgm * yseg;
  const int yb = min(g.ny, ya + yseg);
  for (int y0 = ya; y0 < yb; y0 += kUY) {
    float2 v[kUY];
#pragma unroll
    for (int u = 0; u < kUY; ++u) v[u] = col[(size_t)min(y0 + u, g.ny - 1) * g.nx];
#pragma unroll
    for (int u = 0; u < kUY; ++u) {
      // rows past the segment end belong to the next segment: weight them by zero
      const float keep = (y0 + u < yb) ? 1.f : 0.f;
      const float2 vv = make_float2(keep * v[u].x, keep * v[u].y);
      const float2* tw = tw_yT + (size_t)(y0 + u) * kyp + j0;
#pragma unroll
      for (int w = 0; w < kJG; ++w) cmac_conj(acc[w], vv, tw[w]);
    }
  }
  if (sgm > 0) {
#pragma unroll
    for (int w = 0; w < kJG; ++w) sh[sgm - 1][w][tx] = acc[w];
  }
  __syncthreads();
  if (sgm == 0 && x < g.nx) {
    float2* dst = H + ((size_t)ch * g.ky + j0) * g.nx + x;
#pragma unroll
    for (int w = 0; w < kJG; ++w) {
      float2 s = acc[w];
#pragma unroll
      for (int o = 0; o < kYS - 1; ++o) {
        s.x += sh[o][w][tx].x;
        s.y += sh[o][w][tx].y;
      }
      if (j0 + w < g.ky) dst[(size_t)w * g.nx] = s;
    }
  }
}

// x stage: one output (kx, row) per column of a 64 x kXS block over the flattened rows
// (c*kzh + h, ky); wavefront s sums a contiguous 1/kXS of x in chunks of kU (H rows and the
// transposed twiddles), the partial sums are added in LDS in a fixed order.
constexpr int kXS = 4;

__global__ __launch_bounds__(64 * kXS) void k_pi_x(Geo g, int rows, int xseg,
                                                   const float2* __restrict__ H,
                                                   const float2* __restrict__ tw_xT,
                                                   float2* __restrict__ P) {
  BL_BATCH(g.bat)
  BL_AT(H, g.bat);
  BL_AT(P, g.bat);
  __shared__ float2 sh[kXS - 1][64];
  const int tx = threadIdx.x;
  const int sgm = wave_uniform(threadIdx.y);
  const int t = blockIdx.x * 64 + tx;
  const int r = t / g.kx;
  const int jx = t - r * g.kx;
  const int rc = r < rows ? r : rows - 1;   // clamped row: loads stay in bounds
  const float2* row = H + (size_t)rc * g.nx;
  const int xa = sgm * xseg;
  const int xb = min(g.nx, xa + xseg);
  float2 a0 = make_float2(0.f, 0.f), a1 = a0;
  for (int x0 = xa; x0 < xb; x0 += kU) {
    float2 hv[kU], tv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float keep = (x0 + u < xb) ? 1.f : 0.f;   // the next segment's columns
      const float2 v = row[min(x0 + u, g.nx - 1)];
      hv[u] = make_float2(keep * v.x, keep * v.y);
      tv[u] = tw_xT[(size_t)(x0 + u) * g.kx + jx];   // zero rows past nx
    }
#pragma unroll
    for (int u = 0; u < kU; u += 2) {
      cmac_conj(a0, hv[u], tv[u]);
      cmac_conj(a1, hv[u + 1], tv[u + 1]);
    }
  }
  float2 acc = make_float2(a0.x + a1.x, a0.y + a1.y);
  if (sgm > 0) sh[sgm - 1][tx] = acc;
  __syncthreads();
  if (sgm == 0 && r < rows) {
#pragma unroll
    for (int o = 0; o < kXS - 1; ++o) {
      acc.x += sh[o][tx].x;
      acc.y += sh[o][tx].y;
    }
    P[(size_t)r * g.kx + jx] = acc;
  }
}

// ---------------------------------------------------------------------------- band kernels
__device__ __forceinline__ void band_index(const Geo& g, int b, int& jx, int& jy, int& jz) {
  const int r = b / g.kx;
  jx = b - r * g.kx;
  jz = r / g.ky;
  jy = r - jz * g.ky;
}
__device__ __forceinline__ bool unpaired(const Geo& g, int jx, int jy, int jz) {
  return jx == 0 || jy == 0 || (g.kz > 1 && jz == 0);
}
__device__ __forceinline__ int mirror(const Geo& g, int jx, int jy, int jz) {
  const int mx = g.kx - jx, my = g.ky - jy, mz = g.kz > 1 ? g.kz - jz : 0;
  return (mz * g.ky + my) * g.kx + mx;
}

// q_c = 2 pi k_c / l_c (l_c = n_c / N_ref): the spectral divergence is i sum_c q_c v~_c
template <int DIM>
__device__ __forceinline__ void div_symbol(const Geo& g, int jx, int jy, int jz, float* q) {
  const float two_pi = 6.283185307179586f;
  const int kv[3] = {jx - g.kx / 2, jy - g.ky / 2, jz - g.kz0};
  const int nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int c = 0; c < DIM; ++c) q[c] = two_pi * (float)kv[c] * ((float)g.nref / (float)nn[c]);
}

// Divergence-free part of one band index of a velocity: o - q (q . o) / |q|^2 (identity at
// k = 0).  Written so that the conjugate-mirror index (q -> -q, o -> conj o) gets exactly the
// conjugate result, which keeps the output Hermitian.
template <int DIM>
__device__ __forceinline__ void leray(const float* q, float2* o) {
  float qq = 0.f;
  float2 s = make_float2(0.f, 0.f);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    qq = fmaf(q[c], q[c], qq);
    s.x = fmaf(q[c], o[c].x, s.x);
    s.y = fmaf(q[c], o[c].y, s.y);
  }
  if (qq > 0.f) {
    const float2 t = make_float2(s.x / qq, s.y / qq);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      o[c].x = fmaf(-q[c], t.x, o[c].x);
      o[c].y = fmaf(-q[c], t.y, o[c].y);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_band_prep(Geo g, const float2* __restrict__ raw,
                                                   float2* __restrict__ out, int with_div,
                                                   const double* __restrict__ Lhat64,
                                                   double* __restrict__ reg_partial,
                                                   double reg_weight, int reg_accumulate,
                                                   size_t nstride) {
  BL_BATCH(g.bat)
  BL_AT(raw, g.bat);
  BL_AT(out, g.bat);
  BL_AT(Lhat64, g.bat);
  BL_AT(reg_partial, g.bat);
  double acc = 0.0;
  const int B = (int)g.B;
  raw += blockIdx.y * nstride;   // node blockIdx.y (nodes > 1 only without the regulariser sum)
  out += blockIdx.y * nstride;
  for (int b = blockIdx.x * 256 + threadIdx.x; b < B; b += gridDim.x * 256) {
    int jx, jy, jz;
    band_index(g, b, jx, jy, jz);
    const bool up = unpaired(g, jx, jy, jz);
    const int mb = up ? b : mirror(g, jx, jy, jz);
    float2 a[DIM], m[DIM], o[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      a[c] = raw[c * B + b];
      m[c] = raw[c * B + mb];
    }
    float q[DIM];
    div_symbol<DIM>(g, jx, jy, jz, q);
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      o[c] = up ? make_float2(0.f, 0.f)
                : make_float2(0.5f * (a[c].x + m[c].x), 0.5f * (a[c].y - m[c].y));
    if (g.gamma) leray<DIM>(q, o);
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[c * B + b] = o[c];
    if (reg_partial) {
      const double l = Lhat64[b];
#pragma unroll
      for (int c = 0; c < DIM; ++c) acc += l * ((double)o[c].x * o[c].x + (double)o[c].y * o[c].y);
    }
    if (with_div) {
      // r~ = sum_c 2 pi i (k_c / l_c) v~_c with l_c = n_c / N_ref
      float2 d = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        d.x = fmaf(-q[c], o[c].y, d.x);
        d.y = fmaf(q[c], o[c].x, d.y);
      }
      out[DIM * B + b] = d;
    }
  }
  if (reg_partial) {
    const double tot = block_reduce_256<false>(acc);
    if (threadIdx.x == 0) {
      const double v = reg_weight == 1.0 ? tot : reg_weight * tot;
      reg_partial[blockIdx.x] = reg_accumulate ? reg_partial[blockIdx.x] + v : v;
    }
  }
}

// One thread per band index, all C components: Hermitian completion from the kz >= 0 half, the
// regulariser term, and (leray) the divergence-free part of the C = dim components.  C is a
// template parameter so that the loads of all components are issued together.
template <int DIM, int C>
__global__ __launch_bounds__(256) void k_band_finalize(Geo g,
                                                       const float2* __restrict__ vproj,
                                                       const float* __restrict__ Lhat,
                                                       const float2* __restrict__ P,
                                                       float scale, float2* __restrict__ out,
                                                       int* __restrict__ nonfinite, int leray_on,
                                                       size_t vstride, size_t pstride,
                                                       size_t ostride,
                                                       const float2* __restrict__ dotp,
                                                       double* __restrict__ dot_part,
                                                       double* __restrict__ sq_part,
                                                       double* __restrict__ max_part) {
  BL_BATCH(g.bat)
  BL_AT(vproj, g.bat);
  BL_AT(Lhat, g.bat);
  BL_AT(P, g.bat);
  BL_AT(out, g.bat);
  BL_AT(nonfinite, g.bat);
  BL_AT(dotp, g.bat);
  BL_AT(dot_part, g.bat);
  BL_AT(sq_part, g.bat);
  BL_AT(max_part, g.bat);
  double dacc = 0.0, sacc = 0.0, macc = 0.0;
  const int B = (int)g.B;
  if (vproj) vproj += blockIdx.y * vstride;   // node blockIdx.y
  P += blockIdx.y * pstride;
  out += blockIdx.y * ostride;
  for (int b = blockIdx.x * 256 + threadIdx.x; b < B; b += gridDim.x * 256) {
    int jx, jy, jz;
    band_index(g, b, jx, jy, jz);
    const bool up = unpaired(g, jx, jy, jz);
    const int kzv = jz - g.kz0;
    // Both half-spectrum entries a component may need, at indices valid for every band index
    // (unpaired ones read entry 0 and are zeroed): the direct entry for kz >= 0, the conjugate
    // mirror for kz <= 0.  All loads are unconditional so that they are in flight together; a
    // load inside a branch waits before the next one.
    const size_t ia = up || kzv < 0 ? 0 : ((size_t)kzv * g.ky + jy) * g.kx + jx;
    const size_t im = up || kzv > 0 ? 0 : ((size_t)(-kzv) * g.ky + (g.ky - jy)) * g.kx + (g.kx - jx);
    const size_t ph = (size_t)g.kzh * g.ky * g.kx;
    float2 va[C], vm[C], vp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      va[c] = P[c * ph + ia];
      vm[c] = P[c * ph + im];
      vp[c] = vproj ? vproj[c * B + b] : make_float2(0.f, 0.f);
    }
    const float l = vproj ? Lhat[b] : 0.f;
    float2 o[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      o[c] = make_float2(0.f, 0.f);
      if (up) continue;
      float2 pv;
      if (kzv > 0) {
        pv = va[c];
      } else if (kzv < 0) {
        pv = make_float2(vm[c].x, -vm[c].y);
      } else {
        // kz = 0 plane: average with the conjugate mirror so the output is exactly Hermitian
        pv = make_float2(0.5f * (va[c].x + vm[c].x), 0.5f * (va[c].y - vm[c].y));
      }
      o[c] = make_float2(scale * pv.x, scale * pv.y);
      if (vproj) {
        o[c].x = fmaf(l, vp[c].x, o[c].x);
        o[c].y = fmaf(l, vp[c].y, o[c].y);
      }
    }
    if constexpr (C == DIM) {
      if (leray_on && !up) {
        float q[DIM];
        div_symbol<DIM>(g, jx, jy, jz, q);
        leray<DIM>(q, o);
      }
    }
    bool bad = false;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      bad = bad || !isfinite(o[c].x) || !isfinite(o[c].y);
      out[c * B + b] = o[c];
    }
    if (bad) *nonfinite = 1;
    if (dot_part) {   // Re conj(dotp) o, the components of this band index in order
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float2 d = dotp[c * B + b];
        dacc = fma((double)d.x, (double)o[c].x, dacc);
        dacc = fma((double)d.y, (double)o[c].y, dacc);
      }
    }
    if (sq_part) {   // |o|^2 and max |o| (the gradient's norms)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sacc = fma((double)o[c].x, (double)o[c].x, sacc);
        sacc = fma((double)o[c].y, (double)o[c].y, sacc);
        macc = fmax(macc, sqrt((double)o[c].x * o[c].x + (double)o[c].y * o[c].y));
      }
    }
  }
  // (the whole block takes these branches: kernel arguments decide)
  if (dot_part) {
    const double r = block_reduce_256<false>(dacc);
    if (threadIdx.x == 0) dot_part[blockIdx.x] = r;
  }
  if (sq_part) {
    const double r = block_reduce_256<false>(sacc);
    if (threadIdx.x == 0) sq_part[blockIdx.x] = r;
    const double m = block_reduce_256<true>(macc);
    if (threadIdx.x == 0) max_part[blockIdx.x] = m;
  }
}

template <int KZH>
void launch_z_pair(const Geo& g, const DftPlan& p, const float2* F2, float* out, int C,
                   const float* f, float2* G, hipStream_t s, bool inverse) {
  const int nq = g.nx * g.ny;
  if (inverse) {
    // split z into chunks so that a launch has enough blocks to fill the chip
    // (z, nz - z) pairs: z = 0 .. nz/2, in chunks of at most 64 (LDS: 64 twiddle rows)
    // split further until the launch has enough blocks to fill the chip
    const int npair = g.nz / 2 + 1;
    const int qblocks = (nq + 255) / 256;
    int nchunk = (npair + 63) / 64;
    while (qblocks * nchunk * C < 768 && nchunk * 8 < npair) nchunk *= 2;
    // launch shape: more z chunks per column (each output's arithmetic is unchanged)
    for (int m = g.zv[TR_IOTA_Z]; m > 1 && nchunk * 4 <= npair; m /= 2) nchunk *= 2;
    const int zchunk = (npair + nchunk - 1) / nchunk;
    nchunk = (npair + zchunk - 1) / zchunk;
    const size_t lds = (size_t)zchunk * (KZH == 1 ? 2 : KZH) * sizeof(float2);
    BL_LAUNCH(k_iota_z<KZH>, batch_grid(dim3(qblocks, nchunk, C), g.bat), dim3(256), lds, s, g,
              F2, p.tw_zT, out, zchunk);
  } else {
    BL_LAUNCH(k_pi_z<KZH>, batch_grid(dim3((nq + 63) / 64, C), g.bat), dim3(64, kNW), 0, s, g,
              f, p.tw_zT, G);
  }
}

void z_stage(const Geo& g, const DftPlan& p, const float2* F2, float* out, int C,
             const float* f, float2* G, hipStream_t s, bool inverse) {
  const int k = g.kzh;
  if (k <= 1) launch_z_pair<1>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 4) launch_z_pair<4>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 8) launch_z_pair<8>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 12) launch_z_pair<12>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 16) launch_z_pair<16>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 20) launch_z_pair<20>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 24) launch_z_pair<24>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 32) launch_z_pair<32>(g, p, F2, out, C, f, G, s, inverse);
  else if (k <= 48) launch_z_pair<48>(g, p, F2, out, C, f, G, s, inverse);
  else launch_z_pair<64>(g, p, F2, out, C, f, G, s, inverse);
}

}  // namespace

void iota_xy(const Geo& g, const DftPlan& p, const float2* band, int C, hipStream_t s) {
  const size_t lds = ((size_t)g.ky * g.kx + (size_t)g.ky * kFX) * sizeof(float2);
  // launch shape 16 or 32: the fused stage with that many rows per block; 0: the two stages
  // (nyp is a multiple of 32: the rows of every block are in the table)
  if (g.zv[TR_IOTA_XY] != 0 && lds <= kFusedLds) {
    const dim3 b(256);
    if (g.zv[TR_IOTA_XY] == 16)
      hipLaunchKernelGGL(k_iota_xy<16>,
                         batch_grid(dim3((g.nx + kFX - 1) / kFX, (g.ny + 15) / 16, C * g.kzh),
                                    g.bat),
                         b, lds, s, g, band, p.tw_x, p.tw_y, p.nyp, p.bufB);
    else
      hipLaunchKernelGGL(k_iota_xy<32>,
                         batch_grid(dim3((g.nx + kFX - 1) / kFX, (g.ny + 31) / 32, C * g.kzh),
                                    g.bat),
                         b, lds, s, g, band, p.tw_x, p.tw_y, p.nyp, p.bufB);
    return;
  }
  const int xb = (g.nx + 63) / 64;
  hipLaunchKernelGGL(k_iota_x, batch_grid(dim3(xb, g.ky, C * g.kzh), g.bat), dim3(64), 0, s, g,
                     band, p.tw_x, p.bufA);
  hipLaunchKernelGGL(k_iota_y, batch_grid(dim3(xb, p.nyp / kYG, C * g.kzh), g.bat), dim3(64), 0,
                     s, g, p.bufA, p.tw_y, p.nyp, p.bufB);
}

void iota_z(const Geo& g, const DftPlan& p, int C, float* out, hipStream_t s) {
  if (p.mixed)
    iota_z_mixed(g, p, p.bufB, C, out, s);
  else
    z_stage(g, p, p.bufB, out, C, nullptr, nullptr, s, true);
}

void iota(const Geo& g, const DftPlan& p, const float2* band, int C, float* out, hipStream_t s) {
  iota_xy(g, p, band, C, s);
  iota_z(g, p, C, out, s);
}

void pi_half(const Geo& g, const DftPlan& p, const float* grid, int C, float2* P, hipStream_t s) {
  pi_z(g, p, grid, C, s);
  pi_yx(g, p, C, P, s);
}

void pi_z(const Geo& g, const DftPlan& p, const float* grid, int C, hipStream_t s) {
  if (p.mixed)
    pi_z_mixed(g, p, grid, C, p.bufA, s);
  else
    z_stage(g, p, nullptr, nullptr, C, grid, p.bufA, s, false);
}

void pi_yx(const Geo& g, const DftPlan& p, int C, float2* P, hipStream_t s) {
  const int xb = (g.nx + 63) / 64;
  const int yseg = ((g.ny + kYS - 1) / kYS + kUY - 1) / kUY * kUY;
  hipLaunchKernelGGL(k_pi_y, batch_grid(dim3(xb, p.kyp / kJG, C * g.kzh), g.bat), dim3(64, kYS),
                     0, s, g, p.bufA, p.tw_yT, p.kyp, yseg, p.bufB);
  const int rows = C * g.kzh * g.ky;
  const int xseg = ((g.nx + kXS - 1) / kXS + kU - 1) / kU * kU;
  hipLaunchKernelGGL(k_pi_x, batch_grid(dim3((rows * g.kx + 63) / 64), g.bat), dim3(64, kXS), 0,
                     s, g, rows, xseg, p.bufB, p.tw_xT, P);
}

void band_prep(const Geo& g, const float2* raw, float2* out, int with_div, const double* Lhat64,
               double* reg_partial, hipStream_t s, double reg_weight, int reg_accumulate) {
  // the regulariser sum needs the fixed kRedBlocks grid; the plain projection one thread per
  // band entry
  const int blocks = reg_partial ? kRedBlocks : (int)((g.B + 255) / 256);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_band_prep<3>, batch_grid(dim3(blocks), g.bat), dim3(256), 0, s, g, raw, out, with_div,
                       Lhat64, reg_partial, reg_weight, reg_accumulate, (size_t)0);
  else if (g.dim == 2)
    hipLaunchKernelGGL(k_band_prep<2>, batch_grid(dim3(blocks), g.bat), dim3(256), 0, s, g, raw, out, with_div,
                       Lhat64, reg_partial, reg_weight, reg_accumulate, (size_t)0);
  else
    hipLaunchKernelGGL(k_band_prep<1>, batch_grid(dim3(blocks), g.bat), dim3(256), 0, s, g, raw, out, with_div,
                       Lhat64, reg_partial, reg_weight, reg_accumulate, (size_t)0);
}

void band_prep_nodes(const Geo& g, const float2* raw, float2* out, int nodes, size_t stride,
                     hipStream_t s) {
  const dim3 grid((unsigned)((g.B + 255) / 256), (unsigned)nodes);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_band_prep<3>, grid, dim3(256), 0, s, g, raw, out, 0, nullptr, nullptr,
                       1.0, 0, stride);
  else
    hipLaunchKernelGGL(k_band_prep<2>, grid, dim3(256), 0, s, g, raw, out, 0, nullptr, nullptr,
                       1.0, 0, stride);
}

int finalize_blocks(const Geo& g) { return (int)std::min<int64_t>(kRedBlocks, (g.B + 255) / 256); }

namespace {
void finalize_launch(const Geo& g, int C, const float2* vproj, size_t vstride, const float* Lhat,
                     const float2* P, size_t pstride, float scale, float2* out, size_t ostride,
                     int nodes, int* nonfinite, hipStream_t s, int leray, const float2* dotp,
                     double* dot_part, double* sq_part, double* max_part) {
  const dim3 blocks((unsigned)finalize_blocks(g), (unsigned)nodes);
  const int on = (leray && g.gamma && C == g.dim) ? 1 : 0;
#define BF_LAUNCH(D, CC)                                                                        \
  hipLaunchKernelGGL((k_band_finalize<D, CC>), batch_grid(blocks, g.bat), dim3(256), 0, s, g,     \
                     vproj, Lhat, P,                                                            \
                     scale, out, nonfinite, on, vstride, pstride, ostride, dotp, dot_part,     \
                     sq_part, max_part)
  if (g.dim == 3) {
    switch (C) {
      case 1: BF_LAUNCH(3, 1); break;
      case 2: BF_LAUNCH(3, 2); break;
      case 3: BF_LAUNCH(3, 3); break;
      default: BF_LAUNCH(3, 4); break;
    }
  } else {
    switch (C) {
      case 1: BF_LAUNCH(2, 1); break;
      case 2: BF_LAUNCH(2, 2); break;
      case 3: BF_LAUNCH(2, 3); break;
      default: BF_LAUNCH(2, 4); break;
    }
  }
#undef BF_LAUNCH
}
}  // namespace

void band_finalize(const Geo& g, int C, const float2* vproj, const float* Lhat,
                   const float2* P, float scale, float2* out, int* nonfinite, hipStream_t s,
                   int leray, const float2* dotp, double* dot_part, double* sq_part,
                   double* max_part) {
  finalize_launch(g, C, vproj, 0, Lhat, P, 0, scale, out, 0, 1, nonfinite, s, leray, dotp,
                  dot_part, sq_part, max_part);
}

void band_finalize_nodes(const Geo& g, int C, const float2* vproj, size_t vstride,
                         const float* Lhat, const float2* P, size_t pstride, float scale,
                         float2* out, size_t ostride, int nodes, int* nonfinite, hipStream_t s,
                         int leray) {
  finalize_launch(g, C, vproj, vstride, Lhat, P, pstride, scale, out, ostride, nodes, nonfinite, s,
                  leray, nullptr, nullptr, nullptr, nullptr);
}

}  // namespace bl
