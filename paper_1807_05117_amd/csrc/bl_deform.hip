// Band-limited deformation state equation (paper Section 3.3; continuous system of Section 2.3).
//
// The band state is the displacement u~ = phi~ - id of the inverse map, stepped by the
// classical fourth-order Runge-Kutta method:  d_t u~ = -v~ - D~u~ * v~,  u~(0) = 0, where
// (D~a * b)_i = sum_j (d~_j a_i) * b_j, d~_j = 2 pi i k_j / l_j and * is the truncated
// convolution.  A truncated convolution of band fields is the band part of the pointwise
// product of their grid values on the product grid (P_j >= 3 K_j / 2 points per axis, where no
// product term aliases into the band): the products run on that small grid between the
// iota / pi transforms of bl_dft.hip, and the kernels here do the band-side algebra of a stage
// and the pointwise products.  The gradient and the Gauss-Newton product use the exact
// transpose of the Runge-Kutta step (per step, backwards, kap4 = h/6 rho,
// kap3 = h/3 rho + h A kap4, kap2 = h/3 rho + h/2 A kap3, kap1 = h/6 rho + h/2 A kap2,
// rho <- rho + A (kap1 + ... + kap4) with A = div~(. * v~)) and sum the integrand
// (I + D~U_s)^T * kap_s: its identity part in the band, its deformation part as one product-grid
// accumulation transformed once at the end.  The image level evaluates I0 and its central-
// difference gradient at the displaced points i + N_ref iota(u~(1)) by d-linear interpolation.
#include "bl_internal.h"

namespace bl {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void bidx(const Geo& g, int b, int& jx, int& jy, int& jz) {
  const int r = b / g.kx;
  jx = b - r * g.kx;
  jz = r / g.ky;
  jy = r - jz * g.ky;
}
__device__ __forceinline__ bool unpaired_index(const Geo& g, int jx, int jy, int jz) {
  return jx == 0 || jy == 0 || (g.kz > 1 && jz == 0);
}

// q_c = 2 pi k_c / l_c with l_c = n_c / N_ref of the image grid (not of the product grid)
template <int DIM>
__device__ __forceinline__ void qvec(const Geo& g, int jx, int jy, int jz, float* q) {
  const float two_pi = 6.283185307179586f;
  const int kv[3] = {jx - g.kx / 2, jy - g.ky / 2, jz - g.kz0};
  const int nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int c = 0; c < DIM; ++c) q[c] = two_pi * (float)kv[c] * ((float)g.nref / (float)nn[c]);
}

// value at band index (jx, jy, jz) of the Hermitian field whose kz >= 0 half is Pc; the kz = 0
// plane is averaged with its conjugate mirror so that the result is exactly Hermitian
__device__ __forceinline__ float2 herm(const Geo& g, const float2* __restrict__ Pc, int jx, int jy,
                                       int jz) {
  const int kzv = jz - g.kz0;
  if (kzv > 0) return Pc[((size_t)kzv * g.ky + jy) * g.kx + jx];
  const size_t mi = ((size_t)(kzv < 0 ? -kzv : 0) * g.ky + (g.ky - jy)) * g.kx + (g.kx - jx);
  const float2 m = Pc[mi];
  if (kzv < 0) return make_float2(m.x, -m.y);
  const float2 a = Pc[(size_t)jy * g.kx + jx];
  return make_float2(0.5f * (a.x + m.x), 0.5f * (a.y - m.y));
}

__device__ __forceinline__ float2 times_iq(float q, float2 a) { return make_float2(-q * a.y, q * a.x); }

template <int DIM>
__device__ __forceinline__ void write_deriv(const Geo& g, int b, const float* q, const float2* w,
                                            float2* __restrict__ DU) {
  const size_t B = (size_t)g.B;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) DU[(size_t)(i * DIM + j) * B + b] = times_iq(q[j], w[i]);
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_deriv(Geo g, const float2* __restrict__ U,
                                                        float2* __restrict__ DU) {
  const int B = (int)g.B;
  for (int b = blockIdx.x * kThreads + threadIdx.x; b < B; b += gridDim.x * kThreads) {
    int jx, jy, jz;
    bidx(g, b, jx, jy, jz);
    float q[DIM];
    qvec<DIM>(g, jx, jy, jz, q);
    float2 w[DIM];
    const bool up = unpaired_index(g, jx, jy, jz);
#pragma unroll
    for (int i = 0; i < DIM; ++i) w[i] = up ? make_float2(0.f, 0.f) : U[(size_t)i * B + b];
    write_deriv<DIM>(g, b, q, w, DU);
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_stage(Geo g, float scaleP,
                                                        const float2* __restrict__ Ph,
                                                        const float2* __restrict__ src,
                                                        const float2* __restrict__ un,
                                                        float2* __restrict__ acc, int st,
                                                        float2* __restrict__ unext,
                                                        float2* __restrict__ DU) {
  const int B = (int)g.B;
  const size_t ps = (size_t)g.kzh * g.ky * g.kx;
  const float h = g.dt;
  const float c = st == 3 ? h : 0.5f * h;
  for (int b = blockIdx.x * kThreads + threadIdx.x; b < B; b += gridDim.x * kThreads) {
    int jx, jy, jz;
    bidx(g, b, jx, jy, jz);
    const bool up = unpaired_index(g, jx, jy, jz);
    float2 w[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      float2 k = make_float2(0.f, 0.f), a = k, u = k;
      if (!up) {
        const float2 cv = herm(g, Ph + i * ps, jx, jy, jz);
        const float2 sv = src[(size_t)i * B + b];
        k = make_float2(-sv.x - scaleP * cv.x, -sv.y - scaleP * cv.y);
        u = un[(size_t)i * B + b];
      }
      if (st == 1) {
        a = k;
      } else {
        const float2 p = acc[(size_t)i * B + b];
        const float f = st == 4 ? 1.f : 2.f;
        a = make_float2(fmaf(f, k.x, p.x), fmaf(f, k.y, p.y));
      }
      if (st < 4) {
        acc[(size_t)i * B + b] = a;
        w[i] = make_float2(fmaf(c, k.x, u.x), fmaf(c, k.y, u.y));
      } else {
        const float s6 = h / 6.f;
        w[i] = make_float2(fmaf(s6, a.x, u.x), fmaf(s6, a.y, u.y));
        unext[(size_t)i * B + b] = w[i];
      }
    }
    if (DU) {
      float q[DIM];
      qvec<DIM>(g, jx, jy, jz, q);
      write_deriv<DIM>(g, b, q, w, DU);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_prod(int64_t MP, const float* __restrict__ DG,
                                                       const float* __restrict__ V,
                                                       const float* __restrict__ DG2,
                                                       const float* __restrict__ V2,
                                                       float* __restrict__ out) {
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < MP;
       x += (int64_t)gridDim.x * kThreads) {
    float v[DIM], v2[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      v[j] = V[j * MP + x];
      v2[j] = DG2 ? V2[j * MP + x] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s = fmaf(DG[(i * DIM + j) * MP + x], v[j], s);
      if (DG2) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) s = fmaf(DG2[(i * DIM + j) * MP + x], v2[j], s);
      }
      out[i * MP + x] = s;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_def_adj_init(Geo g, const float2* __restrict__ rho,
                                                           float2* __restrict__ kap,
                                                           float2* __restrict__ Ksum) {
  const int64_t n = (int64_t)g.dim * g.B;
  const float s6 = g.dt / 6.f;
  for (int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * kThreads) {
    const float2 r = rho[b];
    const float2 k = make_float2(s6 * r.x, s6 * r.y);
    kap[b] = k;
    Ksum[b] = k;
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_adj_prod(int64_t MP, const float* __restrict__ KG,
                                                           const float* __restrict__ V,
                                                           const float* __restrict__ DUG,
                                                           float* __restrict__ KV,
                                                           float* __restrict__ GACC, int first) {
  for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < MP;
       x += (int64_t)gridDim.x * kThreads) {
    float kg[DIM], v[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      kg[i] = KG[i * MP + x];
      v[i] = V[i * MP + x];
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) KV[(i * DIM + j) * MP + x] = kg[i] * v[j];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      float s = first ? 0.f : GACC[j * MP + x];
#pragma unroll
      for (int i = 0; i < DIM; ++i) s = fmaf(DUG[(i * DIM + j) * MP + x], kg[i], s);
      GACC[j * MP + x] = s;
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_adj_combine(Geo g, float scaleP,
                                                              const float2* __restrict__ Ph,
                                                              float2* __restrict__ rho,
                                                              float2* __restrict__ Asum,
                                                              float2* __restrict__ Ksum,
                                                              float2* __restrict__ kap, int st,
                                                              int more) {
  const int B = (int)g.B;
  const size_t ps = (size_t)g.kzh * g.ky * g.kx;
  const float h = g.dt;
  // coefficients of the next kap: (rho, A) weights for st = 4, 3, 2
  const float cr = st == 2 ? h / 6.f : h / 3.f;
  const float ca = st == 4 ? h : 0.5f * h;
  for (int b = blockIdx.x * kThreads + threadIdx.x; b < B; b += gridDim.x * kThreads) {
    int jx, jy, jz;
    bidx(g, b, jx, jy, jz);
    const bool up = unpaired_index(g, jx, jy, jz);
    float q[DIM];
    qvec<DIM>(g, jx, jy, jz, q);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const size_t o = (size_t)i * B + b;
      float2 A = make_float2(0.f, 0.f);
      if (!up) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const float2 p = herm(g, Ph + (size_t)(i * DIM + j) * ps, jx, jy, jz);
          const float2 t = times_iq(q[j], p);
          A.x = fmaf(scaleP, t.x, A.x);
          A.y = fmaf(scaleP, t.y, A.y);
        }
      }
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
        if (!more) continue;
        kp = make_float2(h / 6.f * rn.x, h / 6.f * rn.y);
      }
      kap[o] = kp;
      const float2 ks = Ksum[o];
      Ksum[o] = make_float2(ks.x + kp.x, ks.y + kp.y);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_out(Geo g, float scaleP,
                                                      const float2* __restrict__ Ph,
                                                      const float2* __restrict__ Ksum,
                                                      const float2* __restrict__ vproj,
                                                      const float* __restrict__ Lhat,
                                                      float2* __restrict__ out,
                                                      int* __restrict__ nonfinite, int leray_on) {
  const int B = (int)g.B;
  const size_t ps = (size_t)g.kzh * g.ky * g.kx;
  for (int b = blockIdx.x * kThreads + threadIdx.x; b < B; b += gridDim.x * kThreads) {
    int jx, jy, jz;
    bidx(g, b, jx, jy, jz);
    const bool up = unpaired_index(g, jx, jy, jz);
    float2 o[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      o[i] = make_float2(0.f, 0.f);
      if (up) continue;
      const float2 p = herm(g, Ph + (size_t)i * ps, jx, jy, jz);
      const float2 k = Ksum[(size_t)i * B + b];
      o[i] = make_float2(fmaf(scaleP, p.x, k.x), fmaf(scaleP, p.y, k.y));
      if (vproj) {
        const float l = Lhat[b];
        const float2 v = vproj[(size_t)i * B + b];
        o[i].x = fmaf(l, v.x, o[i].x);
        o[i].y = fmaf(l, v.y, o[i].y);
      }
    }
    if (leray_on && !up) {
      // divergence-free part: o - q (q . o) / |q|^2, identity at k = 0
      float q[DIM];
      qvec<DIM>(g, jx, jy, jz, q);
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
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      if (!isfinite(o[i].x) || !isfinite(o[i].y)) *nonfinite = 1;
      out[(size_t)i * B + b] = o[i];
    }
  }
}

// ----------------------------------------------------------------------------- image level
__device__ __forceinline__ int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__global__ __launch_bounds__(kThreads) void k_def_ig4(Geo g, const float* __restrict__ I0,
                                                      float4* __restrict__ IG) {
  const int64_t M = g.M;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    const int x = (int)(v % g.nx);
    const int64_t r = v / g.nx;
    const int y = (int)(r % g.ny);
    const int z = (int)(r / g.ny);
    const int64_t row = (int64_t)g.nx, plane = (int64_t)g.nx * g.ny;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
    const int64_t base = v - x - (int64_t)y * row;   // start of plane z
    float4 o;
    o.x = I0[v];
    o.y = (I0[base + y * row + xp] - I0[base + y * row + xm]) * g.half_nref;
    o.z = (I0[base + yp * row + x] - I0[base + ym * row + x]) * g.half_nref;
    if (g.dim == 3) {
      const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z + 1 == g.nz ? 0 : z + 1;
      o.w = (I0[zp * plane + y * row + x] - I0[zm * plane + y * row + x]) * g.half_nref;
    } else {
      o.w = 0.f;
    }
    IG[v] = o;
  }
}

// offset in voxels: non-finite -> 0, magnitudes beyond 2^20 clamped (any such field is far
// outside the method's range; the clamp only keeps the index arithmetic in int range)
__device__ __forceinline__ float sane_offset(float o) {
  if (!(o == o)) return 0.f;
  return fminf(fmaxf(o, -1048576.f), 1048576.f);
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_warp(Geo g, const float* __restrict__ UG,
                                                       const float4* __restrict__ IG,
                                                       float* __restrict__ m1,
                                                       float4* __restrict__ GP) {
  const int64_t M = g.M;
  const float nref = (float)g.nref;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    const int c0[3] = {(int)(v % g.nx), (int)((v / g.nx) % g.ny), (int)(v / ((int64_t)g.nx * g.ny))};
    const int nn[3] = {g.nx, g.ny, g.nz};
    int i0[3] = {0, 0, 0}, i1[3] = {0, 0, 0};
    float fr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const float p = (float)c0[j] + sane_offset(nref * UG[j * M + v]);
      const float f = floorf(p);
      fr[j] = p - f;
      i0[j] = wrap_index((int)f, nn[j]);
      i1[j] = i0[j] + 1 == nn[j] ? 0 : i0[j] + 1;
    }
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t row = g.nx, plane = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
      float w = 1.f;
      int64_t idx = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const int bit = (corner >> j) & 1;
        w *= bit ? fr[j] : 1.f - fr[j];
        const int ij = bit ? i1[j] : i0[j];
        idx += (j == 0 ? 1 : (j == 1 ? row : plane)) * (int64_t)ij;
      }
      const float4 s = IG[idx];
      acc.x = fmaf(w, s.x, acc.x);
      acc.y = fmaf(w, s.y, acc.y);
      acc.z = fmaf(w, s.z, acc.z);
      acc.w = fmaf(w, s.w, acc.w);
    }
    m1[v] = acc.x;
    GP[v] = make_float4(acc.y, acc.z, acc.w, 0.f);
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_rho1(Geo g, const float* __restrict__ m1,
                                                       const float* __restrict__ I1,
                                                       const float4* __restrict__ GP,
                                                       float* __restrict__ Bf) {
  const int64_t M = g.M;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    const float lam = g.lam_scale * (m1[v] - I1[v]);
    const float4 gp = GP[v];
    Bf[v] = lam * gp.x;
    Bf[M + v] = lam * gp.y;
    if (DIM == 3) Bf[2 * M + v] = lam * gp.z;
  }
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_def_drho1(Geo g, const float* __restrict__ DU,
                                                        const float4* __restrict__ GP,
                                                        float* __restrict__ Bf) {
  const int64_t M = g.M;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < M;
       v += (int64_t)gridDim.x * kThreads) {
    const float4 gp = GP[v];
    float dm = gp.x * DU[v];
    dm = fmaf(gp.y, DU[M + v], dm);
    if (DIM == 3) dm = fmaf(gp.z, DU[2 * M + v], dm);
    const float dl = g.lam_scale * dm;
    Bf[v] = dl * gp.x;
    Bf[M + v] = dl * gp.y;
    if (DIM == 3) Bf[2 * M + v] = dl * gp.z;
  }
}

int blocks_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

}  // namespace

#define DIM_DISPATCH(KERNEL, BLOCKS, ...)                                                 \
  do {                                                                                    \
    if (g.dim == 3)                                                                       \
      hipLaunchKernelGGL(KERNEL<3>, dim3(BLOCKS), dim3(kThreads), 0, s, __VA_ARGS__);     \
    else                                                                                  \
      hipLaunchKernelGGL(KERNEL<2>, dim3(BLOCKS), dim3(kThreads), 0, s, __VA_ARGS__);     \
  } while (0)

void def_deriv(const Geo& g, const float2* U, float2* DU, hipStream_t s) {
  DIM_DISPATCH(k_def_deriv, blocks_for(g.B), g, U, DU);
}

void def_stage(const Geo& g, float scaleP, const float2* Ph, const float2* src, const float2* un,
               float2* acc, int st, float2* unext, float2* DU, hipStream_t s) {
  DIM_DISPATCH(k_def_stage, blocks_for(g.B), g, scaleP, Ph, src, un, acc, st, unext, DU);
}

void def_prod(const Geo& g, int64_t MP, const float* DG, const float* V, const float* DG2,
              const float* V2, float* out, hipStream_t s) {
  DIM_DISPATCH(k_def_prod, blocks_for(MP), MP, DG, V, DG2, V2, out);
}

void def_adj_init(const Geo& g, const float2* rho, float2* kap, float2* Ksum, hipStream_t s) {
  hipLaunchKernelGGL(k_def_adj_init, dim3(blocks_for((int64_t)g.dim * g.B)), dim3(kThreads), 0, s,
                     g, rho, kap, Ksum);
}

void def_adj_prod(const Geo& g, int64_t MP, const float* KG, const float* V, const float* DUG,
                  float* KV, float* GACC, int first, hipStream_t s) {
  DIM_DISPATCH(k_def_adj_prod, blocks_for(MP), MP, KG, V, DUG, KV, GACC, first);
}

void def_adj_combine(const Geo& g, float scaleP, const float2* Ph, float2* rho, float2* Asum,
                     float2* Ksum, float2* kap, int st, int more, hipStream_t s) {
  DIM_DISPATCH(k_def_adj_combine, blocks_for(g.B), g, scaleP, Ph, rho, Asum, Ksum, kap, st, more);
}

void def_out(const Geo& g, float scaleP, const float2* Ph, const float2* Ksum,
             const float2* vproj, const float* Lhat, float2* out, int* nonfinite, hipStream_t s) {
  const int on = g.gamma ? 1 : 0;
  DIM_DISPATCH(k_def_out, blocks_for(g.B), g, scaleP, Ph, Ksum, vproj, Lhat, out, nonfinite, on);
}

void def_ig4(const Geo& g, const float* I0, float4* IG, hipStream_t s) {
  hipLaunchKernelGGL(k_def_ig4, dim3(blocks_for(g.M)), dim3(kThreads), 0, s, g, I0, IG);
}

void def_warp(const Geo& g, const float* UG, const float4* IG, float* m1, float4* GP,
              hipStream_t s) {
  DIM_DISPATCH(k_def_warp, blocks_for(g.M), g, UG, IG, m1, GP);
}

void def_rho1(const Geo& g, const float* m1, const float* I1, const float4* GP, float* Bf,
              hipStream_t s) {
  DIM_DISPATCH(k_def_rho1, blocks_for(g.M), g, m1, I1, GP, Bf);
}

void def_drho1(const Geo& g, const float* DU, const float4* GP, float* Bf, hipStream_t s) {
  DIM_DISPATCH(k_def_drho1, blocks_for(g.M), g, DU, GP, Bf);
}

}  // namespace bl
