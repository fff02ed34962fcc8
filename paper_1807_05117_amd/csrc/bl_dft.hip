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

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
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

// ---------------------------------------------------------------------------- iota stages
__global__ __launch_bounds__(64) void k_iota_x(Geo g, const float2* __restrict__ band,
                                               const float2* __restrict__ tw_x,
                                               float2* __restrict__ F1) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int jy = blockIdx.y;
  const int ch = blockIdx.z;
  if (x >= g.nx) return;
  const int c = ch / g.kzh, h = ch - c * g.kzh;
  const float2* row = band + ((size_t)(c * g.kz + g.kz0 + h) * g.ky + jy) * g.kx;
  float2 acc = make_float2(0.f, 0.f);
  for (int jx = 0; jx < g.kx; ++jx) cmac(acc, row[jx], tw_x[(size_t)jx * g.nx + x]);
  F1[((size_t)ch * g.ky + jy) * g.nx + x] = acc;
}

__global__ __launch_bounds__(64) void k_iota_y(Geo g, const float2* __restrict__ F1,
                                               const float2* __restrict__ tw_y,
                                               float2* __restrict__ F2) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y;
  const int ch = blockIdx.z;
  if (x >= g.nx) return;
  const float2* col = F1 + (size_t)ch * g.ky * g.nx + x;
  float2 acc = make_float2(0.f, 0.f);
  for (int jy = 0; jy < g.ky; ++jy) cmac(acc, col[(size_t)jy * g.nx], tw_y[(size_t)jy * g.ny + y]);
  F2[((size_t)ch * g.ny + y) * g.nx + x] = acc;
}

template <int KZH>
__global__ __launch_bounds__(256) void k_iota_z(Geo g, const float2* __restrict__ F2,
                                                const float2* __restrict__ tw_z,
                                                float* __restrict__ out, int zchunk) {
  const int nq = g.nx * g.ny;
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.z;
  if (q >= nq) return;
  float2 f[KZH];
  const float2* src = F2 + (size_t)c * g.kzh * nq + q;
#pragma unroll
  for (int h = 0; h < KZH; ++h) {
    float2 v = h < g.kzh ? src[(size_t)h * nq] : make_float2(0.f, 0.f);
    if (h > 0) { v.x *= 2.f; v.y *= 2.f; }
    f[h] = v;
  }
  const int z0 = blockIdx.y * zchunk;
  const int z1 = min(g.nz, z0 + zchunk);
  float* dst = out + (size_t)c * g.M + q;
  for (int z = z0; z < z1; ++z) {
    float acc0 = f[0].x, acc1 = 0.f;
#pragma unroll
    for (int h = 1; h < KZH; ++h) {
      const float2 t = tw_z[(size_t)h * g.nz + z];
      acc0 = fmaf(f[h].x, t.x, acc0);
      acc1 = fmaf(-f[h].y, t.y, acc1);
    }
    dst[(size_t)z * nq] = acc0 + acc1;
  }
}

// ------------------------------------------------------------------------------ pi stages
template <int KZH>
__global__ __launch_bounds__(256) void k_pi_z(Geo g, const float* __restrict__ f,
                                              const float2* __restrict__ tw_z,
                                              float2* __restrict__ G) {
  constexpr int CH = (KZH % 8 == 0) ? 8 : ((KZH % 4 == 0) ? 4 : 1);
  __shared__ float2 sh[3][CH][64];
  const int nq = g.nx * g.ny;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int q = blockIdx.x * 64 + tx;
  const int c = blockIdx.y;
  float2 acc[KZH];
#pragma unroll
  for (int h = 0; h < KZH; ++h) acc[h] = make_float2(0.f, 0.f);
  if (q < nq) {
    const float* src = f + (size_t)c * g.M + q;
    for (int z = ty; z < g.nz; z += 4) {
      const float v = src[(size_t)z * nq];
#pragma unroll
      for (int h = 0; h < KZH; ++h) {
        const float2 t = tw_z[(size_t)h * g.nz + z];
        acc[h].x = fmaf(v, t.x, acc[h].x);
        acc[h].y = fmaf(-v, t.y, acc[h].y);
      }
    }
  }
#pragma unroll
  for (int h0 = 0; h0 < KZH; h0 += CH) {
    if (ty > 0) {
#pragma unroll
      for (int hh = 0; hh < CH; ++hh) sh[ty - 1][hh][tx] = acc[h0 + hh];
    }
    __syncthreads();
    if (ty == 0) {
#pragma unroll
      for (int hh = 0; hh < CH; ++hh) {
        acc[h0 + hh].x += (sh[0][hh][tx].x + sh[1][hh][tx].x) + sh[2][hh][tx].x;
        acc[h0 + hh].y += (sh[0][hh][tx].y + sh[1][hh][tx].y) + sh[2][hh][tx].y;
      }
    }
    __syncthreads();
  }
  if (ty == 0 && q < nq) {
    float2* dst = G + (size_t)c * g.kzh * nq + q;
#pragma unroll
    for (int h = 0; h < KZH; ++h)
      if (h < g.kzh) dst[(size_t)h * nq] = acc[h];
  }
}

__global__ __launch_bounds__(64) void k_pi_y(Geo g, const float2* __restrict__ G,
                                             const float2* __restrict__ tw_y,
                                             float2* __restrict__ H) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int jy = blockIdx.y;
  const int ch = blockIdx.z;
  if (x >= g.nx) return;
  const float2* col = G + (size_t)ch * g.ny * g.nx + x;
  const float2* tw = tw_y + (size_t)jy * g.ny;
  float2 acc = make_float2(0.f, 0.f);
  for (int y = 0; y < g.ny; ++y) cmac_conj(acc, col[(size_t)y * g.nx], tw[y]);
  H[((size_t)ch * g.ky + jy) * g.nx + x] = acc;
}

__global__ __launch_bounds__(64) void k_pi_x(Geo g, const float2* __restrict__ H,
                                             const float2* __restrict__ tw_x,
                                             float2* __restrict__ P) {
  const int jx = blockIdx.x * 64 + threadIdx.x;
  const int jy = blockIdx.y;
  const int ch = blockIdx.z;
  if (jx >= g.kx) return;
  const float2* row = H + ((size_t)ch * g.ky + jy) * g.nx;
  const float2* tw = tw_x + (size_t)jx * g.nx;
  float2 acc = make_float2(0.f, 0.f);
  for (int x = 0; x < g.nx; ++x) cmac_conj(acc, row[x], tw[x]);
  P[((size_t)ch * g.ky + jy) * g.kx + jx] = acc;
}

// ---------------------------------------------------------------------------- band kernels
__device__ __forceinline__ void band_index(const Geo& g, int64_t b, int& jx, int& jy, int& jz) {
  jx = (int)(b % g.kx);
  const int64_t r = b / g.kx;
  jy = (int)(r % g.ky);
  jz = (int)(r / g.ky);
}
__device__ __forceinline__ bool unpaired(const Geo& g, int jx, int jy, int jz) {
  return jx == 0 || jy == 0 || (g.kz > 1 && jz == 0);
}
__device__ __forceinline__ int64_t mirror(const Geo& g, int jx, int jy, int jz) {
  const int mx = g.kx - jx, my = g.ky - jy, mz = g.kz > 1 ? g.kz - jz : 0;
  return ((int64_t)mz * g.ky + my) * g.kx + mx;
}

__global__ __launch_bounds__(256) void k_band_prep(Geo g, const float2* __restrict__ raw,
                                                   float2* __restrict__ out, int with_div,
                                                   const double* __restrict__ Lhat64,
                                                   double* __restrict__ reg_partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < g.B;
       b += (int64_t)gridDim.x * 256) {
    int jx, jy, jz;
    band_index(g, b, jx, jy, jz);
    const bool up = unpaired(g, jx, jy, jz);
    const int64_t mb = up ? b : mirror(g, jx, jy, jz);
    float2 o[3];
    for (int c = 0; c < g.dim; ++c) {
      if (up) {
        o[c] = make_float2(0.f, 0.f);
      } else {
        const float2 a = raw[c * g.B + b], m = raw[c * g.B + mb];
        o[c] = make_float2(0.5f * (a.x + m.x), 0.5f * (a.y - m.y));
      }
      out[c * g.B + b] = o[c];
      if (reg_partial) acc += Lhat64[b] * ((double)o[c].x * o[c].x + (double)o[c].y * o[c].y);
    }
    if (with_div) {
      // r~ = sum_c 2 pi i (k_c / l_c) v~_c with l_c = n_c / N_ref
      const float two_pi = 6.283185307179586f;
      const int kv[3] = {jx - g.kx / 2, jy - g.ky / 2, jz - g.kz0};
      const int nn[3] = {g.nx, g.ny, g.nz};
      float2 d = make_float2(0.f, 0.f);
      for (int c = 0; c < g.dim; ++c) {
        const float qc = two_pi * (float)kv[c] * ((float)g.nref / (float)nn[c]);
        d.x = fmaf(-qc, o[c].y, d.x);
        d.y = fmaf(qc, o[c].x, d.y);
      }
      out[g.dim * g.B + b] = d;
    }
  }
  if (reg_partial) {
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) reg_partial[blockIdx.x] = sh[0];
  }
}

__global__ __launch_bounds__(256) void k_band_finalize(Geo g, int C,
                                                       const float2* __restrict__ vproj,
                                                       const float* __restrict__ Lhat,
                                                       const float2* __restrict__ P,
                                                       float scale, float2* __restrict__ out,
                                                       int* __restrict__ nonfinite) {
  const int64_t total = (int64_t)C * g.B;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int c = (int)(i / g.B);
    const int64_t b = i - (int64_t)c * g.B;
    int jx, jy, jz;
    band_index(g, b, jx, jy, jz);
    float2 o = make_float2(0.f, 0.f);
    if (!unpaired(g, jx, jy, jz)) {
      const int kzv = jz - g.kz0;
      const float2* Pc = P + (size_t)c * g.kzh * g.ky * g.kx;
      float2 pv;
      if (kzv > 0) {
        pv = Pc[((size_t)kzv * g.ky + jy) * g.kx + jx];
      } else if (kzv < 0) {
        const float2 m = Pc[((size_t)(-kzv) * g.ky + (g.ky - jy)) * g.kx + (g.kx - jx)];
        pv = make_float2(m.x, -m.y);
      } else {
        // kz = 0 plane: average with the conjugate mirror so the output is exactly Hermitian
        const float2 a = Pc[(size_t)jy * g.kx + jx];
        const float2 m = Pc[(size_t)(g.ky - jy) * g.kx + (g.kx - jx)];
        pv = make_float2(0.5f * (a.x + m.x), 0.5f * (a.y - m.y));
      }
      o = make_float2(scale * pv.x, scale * pv.y);
      if (vproj) {
        const float l = Lhat[b];
        const float2 v = vproj[(size_t)c * g.B + b];
        o.x = fmaf(l, v.x, o.x);
        o.y = fmaf(l, v.y, o.y);
      }
      if (!isfinite(o.x) || !isfinite(o.y)) *nonfinite = 1;
    }
    out[i] = o;
  }
}

template <int KZH>
void launch_z_pair(const Geo& g, const DftPlan& p, const float2* F2, float* out, int C,
                   const float* f, float2* G, hipStream_t s, bool inverse) {
  const int nq = g.nx * g.ny;
  if (inverse) {
    // split z into chunks so that a launch has enough blocks to fill the chip
    const int qblocks = (nq + 255) / 256;
    int nchunk = 1;
    while (qblocks * nchunk * C < 2048 && nchunk < g.nz) nchunk *= 2;
    const int zchunk = (g.nz + nchunk - 1) / nchunk;
    nchunk = (g.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL(k_iota_z<KZH>, dim3(qblocks, nchunk, C), dim3(256), 0, s, g, F2,
                       p.tw_z, out, zchunk);
  } else {
    hipLaunchKernelGGL(k_pi_z<KZH>, dim3((nq + 63) / 64, C), dim3(64, 4), 0, s, g, f, p.tw_z, G);
  }
}

void z_stage(const Geo& g, const DftPlan& p, const float2* F2, float* out, int C,
             const float* f, float2* G, hipStream_t s, bool inverse) {
  const int k = g.kzh;
  if (k <= 1) launch_z_pair<1>(g, p, F2, out, C, f, G, s, inverse);
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

void iota(const Geo& g, const DftPlan& p, const float2* band, int C, float* out, hipStream_t s) {
  const int xb = (g.nx + 63) / 64;
  hipLaunchKernelGGL(k_iota_x, dim3(xb, g.ky, C * g.kzh), dim3(64), 0, s, g, band, p.tw_x, p.bufA);
  hipLaunchKernelGGL(k_iota_y, dim3(xb, g.ny, C * g.kzh), dim3(64), 0, s, g, p.bufA, p.tw_y, p.bufB);
  z_stage(g, p, p.bufB, out, C, nullptr, nullptr, s, true);
}

void pi_half(const Geo& g, const DftPlan& p, const float* grid, int C, float2* P, hipStream_t s) {
  const int xb = (g.nx + 63) / 64;
  z_stage(g, p, nullptr, nullptr, C, grid, p.bufA, s, false);
  hipLaunchKernelGGL(k_pi_y, dim3(xb, g.ky, C * g.kzh), dim3(64), 0, s, g, p.bufA, p.tw_y, p.bufB);
  hipLaunchKernelGGL(k_pi_x, dim3((g.kx + 63) / 64, g.ky, C * g.kzh), dim3(64), 0, s, g, p.bufB,
                     p.tw_x, P);
}

void band_prep(const Geo& g, const float2* raw, float2* out, int with_div, const double* Lhat64,
               double* reg_partial, hipStream_t s) {
  hipLaunchKernelGGL(k_band_prep, dim3(kRedBlocks), dim3(256), 0, s, g, raw, out, with_div,
                     Lhat64, reg_partial);
}

void band_finalize(const Geo& g, int C, const float2* vproj, const float* Lhat,
                   const float2* P, float scale, float2* out, int* nonfinite, hipStream_t s) {
  const int64_t total = (int64_t)C * g.B;
  const int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_band_finalize, dim3(blocks), dim3(256), 0, s, g, C, vproj, Lhat, P,
                     scale, out, nonfinite);
}

}  // namespace bl
