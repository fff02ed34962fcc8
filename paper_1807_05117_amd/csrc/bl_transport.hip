// Semi-Lagrangian transports of the state, adjoint, incremental state and incremental
// adjoint, the departure-point setup and the body-force accumulation.
//
// Discretisation (paper Section 2.2 equations StateEquation and FirstOrder1-4, the
// commented incremental system of Section 2.2, Section 3.2 with iota(v~)):
//   u = dt * N_ref * v                      velocity in voxels per step
//   X = -(u + Interp(u, i - u)) / 2         forward characteristic (Heun)
//   Y = +(u + Interp(u, i + u)) / 2         backward characteristic (Heun)
//   a = 1 + dt/2 [R + (1 + dt R) r],  R = Interp(r, i + Y),  r = div v
//   m^{n+1} = Interp(m^n, i + X)
//   lambda^n = a Interp(lambda^{n+1}, i + Y),  b = sum_n w_n lambda^n grad m^n
//   t^0 = dt/2 f^0, t^{n+1} = Interp(t^n, i + X) + dt f^{n+1},
//   dm^Nt = Interp(t^{Nt-1}, i + X) + dt/2 f^Nt,  f^n = -grad m^n . dv
// with periodic d-linear interpolation, central differences grad f = (f(i+e) - f(i-e)) N_ref/2
// and trapezoid weights w_n in time.
//
// Layout: every grid field is float32 with x fastest; vector fields are `dim` consecutive
// planes of M floats.  One thread per voxel, 64 x 4 threads per block along (x, y), one
// grid layer of blocks per z plane, so wavefronts read and write whole x rows.
#include "bl_internal.h"

namespace bl {
namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ int wrap(int i, int n) {
  if ((unsigned)i < (unsigned)n) return i;
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Split an offset into the lower cell index (periodic) and the fractional weight.  Offsets
// are clamped to +-2^20 voxels and non-finite offsets are mapped to 0, so every index that
// reaches memory lies in [0, n).
__device__ __forceinline__ void split(float o, int base, int n, int& i0, int& i1, float& w) {
  if (!(fabsf(o) <= 1048576.0f)) o = 0.0f;
  const float f = floorf(o);
  w = o - f;
  i0 = wrap(base + (int)f, n);
  i1 = (i0 + 1 == n) ? 0 : i0 + 1;
}

// All in-volume indices are 32-bit (the host guarantees prod(n) <= 2^30); plane offsets are
// applied to the base pointers.
template <int DIM>
struct Tap {
  uint32_t r00, r01, r10, r11;  // row starts (z0,y0) (z0,y1) (z1,y0) (z1,y1)
  int x0, x1;
  float wx, wy, wz;
};

template <int DIM>
__device__ __forceinline__ Tap<DIM> make_tap(const Geo& g, int x, int y, int z, float ox,
                                             float oy, float oz) {
  Tap<DIM> t;
  int y0, y1;
  split(ox, x, g.nx, t.x0, t.x1, t.wx);
  split(oy, y, g.ny, y0, y1, t.wy);
  if (DIM == 3) {
    int z0, z1;
    split(oz, z, g.nz, z0, z1, t.wz);
    t.r00 = ((uint32_t)z0 * g.ny + y0) * g.nx;
    t.r01 = ((uint32_t)z0 * g.ny + y1) * g.nx;
    t.r10 = ((uint32_t)z1 * g.ny + y0) * g.nx;
    t.r11 = ((uint32_t)z1 * g.ny + y1) * g.nx;
  } else {
    t.wz = 0.0f;
    t.r00 = (uint32_t)y0 * g.nx;
    t.r01 = (uint32_t)y1 * g.nx;
    t.r10 = t.r00;
    t.r11 = t.r01;
  }
  return t;
}

template <int DIM>
__device__ __forceinline__ float apply(const float* __restrict__ f, const Tap<DIM>& t) {
  const float a0 = f[t.r00 + t.x0], a1 = f[t.r00 + t.x1];
  const float b0 = f[t.r01 + t.x0], b1 = f[t.r01 + t.x1];
  const float ra = fmaf(t.wx, a1 - a0, a0);
  const float rb = fmaf(t.wx, b1 - b0, b0);
  const float pa = fmaf(t.wy, rb - ra, ra);
  if (DIM == 2) return pa;
  const float c0 = f[t.r10 + t.x0], c1 = f[t.r10 + t.x1];
  const float d0 = f[t.r11 + t.x0], d1 = f[t.r11 + t.x1];
  const float rc = fmaf(t.wx, c1 - c0, c0);
  const float rd = fmaf(t.wx, d1 - d0, d0);
  const float pb = fmaf(t.wy, rd - rc, rc);
  return fmaf(t.wz, pb - pa, pa);
}

// Central differences of f at voxel (x, y, z), scaled by N_ref / 2.
template <int DIM>
__device__ __forceinline__ void grad_c(const Geo& g, const float* __restrict__ f, int x, int y,
                                       int z, uint32_t p, float* gr) {
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
  const uint32_t row = p - x;
  gr[0] = (f[row + xp] - f[row + xm]) * g.half_nref;
  const uint32_t sy = g.nx;
  const uint32_t pym = y == 0 ? p + (uint32_t)(g.ny - 1) * sy : p - sy;
  const uint32_t pyp = y + 1 == g.ny ? p - (uint32_t)(g.ny - 1) * sy : p + sy;
  gr[1] = (f[pyp] - f[pym]) * g.half_nref;
  if (DIM == 3) {
    const uint32_t sz = (uint32_t)g.nx * g.ny;
    const uint32_t pzm = z == 0 ? p + (uint32_t)(g.nz - 1) * sz : p - sz;
    const uint32_t pzp = z + 1 == g.nz ? p - (uint32_t)(g.nz - 1) * sz : p + sz;
    gr[2] = (f[pzp] - f[pzm]) * g.half_nref;
  }
}

// Kernels that take ZV voxels per thread along z: z is clamped to the grid so that every load
// stays in bounds and the ZV voxels' loads can be issued together; only the stores are
// guarded.
#define VOXEL_XY                                         \
  const int x = blockIdx.x * BX + threadIdx.x;           \
  const int y = blockIdx.y * BY + threadIdx.y;           \
  if (x >= g.nx || y >= g.ny) return;                    \
  const size_t M = (size_t)g.M;                          \
  (void)M;
#define VOXEL_Z(zz)                                      \
  const int zr = blockIdx.z * ZV + (zz);                 \
  const int z = zr < g.nz ? zr : g.nz - 1;               \
  const bool live = zr < g.nz;                           \
  const uint32_t p = ((uint32_t)z * g.ny + y) * g.nx + x;\
  (void)live;

#define VOXEL_PROLOGUE                                   \
  const int x = blockIdx.x * BX + threadIdx.x;           \
  const int y = blockIdx.y * BY + threadIdx.y;           \
  const int z = blockIdx.z;                              \
  if (x >= g.nx || y >= g.ny) return;                    \
  const uint32_t p = ((uint32_t)z * g.ny + y) * g.nx + x; \
  const size_t M = (size_t)g.M;                          \
  (void)M;

template <int DIM>
__global__ __launch_bounds__(BX* BY) void k_setup(Geo g, const float* __restrict__ v,
                                                  float* __restrict__ X, float* __restrict__ Y,
                                                  float* __restrict__ A) {
  VOXEL_PROLOGUE
  const float s = g.dt * (float)g.nref;
  float u[3] = {0.f, 0.f, 0.f};
  for (int c = 0; c < DIM; ++c) u[c] = s * v[c * M + p];
  // forward: X = -(u + Interp(u, i - u)) / 2
  const Tap<DIM> tf = make_tap<DIM>(g, x, y, z, -u[0], -u[1], -u[2]);
  // backward: Y = +(u + Interp(u, i + u)) / 2
  const Tap<DIM> tb = make_tap<DIM>(g, x, y, z, u[0], u[1], u[2]);
  float yo[3] = {0.f, 0.f, 0.f};
  for (int c = 0; c < DIM; ++c) {
    const float* vc = v + c * M;
    const float uf = s * apply<DIM>(vc, tf);
    const float ub = s * apply<DIM>(vc, tb);
    X[c * M + p] = -0.5f * (u[c] + uf);
    yo[c] = 0.5f * (u[c] + ub);
    Y[c * M + p] = yo[c];
  }
  // reaction factor of the adjoint along the backward characteristic (Heun)
  const float* r = v + DIM * M;
  const Tap<DIM> ty = make_tap<DIM>(g, x, y, z, yo[0], yo[1], yo[2]);
  const float R = apply<DIM>(r, ty);
  const float ri = r[p];
  A[p] = 1.0f + 0.5f * g.dt * (R + (1.0f + g.dt * R) * ri);
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* BY) void k_state_step(Geo g, const float* __restrict__ m_in,
                                                       const float* __restrict__ X,
                                                       float* __restrict__ m_out) {
  VOXEL_XY
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    VOXEL_Z(zz)
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    const float v = apply<DIM>(m_in, make_tap<DIM>(g, x, y, z, ox, oy, oz));
    if (live) m_out[p] = v;
  }
}

template <int DIM>
__global__ __launch_bounds__(BX* BY) void k_terminal(Geo g, const float* __restrict__ mT,
                                                     const float* __restrict__ I1,
                                                     float* __restrict__ lam) {
  VOXEL_PROLOGUE
  lam[p] = g.lam_scale * (mT[p] - I1[p]);
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* BY) void k_adj_step(Geo g, const float* __restrict__ lam_in,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ A,
                                                     float* __restrict__ lam_out) {
  VOXEL_XY
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    VOXEL_Z(zz)
    const float ox = Y[p], oy = Y[M + p], oz = DIM == 3 ? Y[2 * M + p] : 0.f;
    const float v = A[p] * apply<DIM>(lam_in, make_tap<DIM>(g, x, y, z, ox, oy, oz));
    if (live) lam_out[p] = v;
  }
}

// b = sum_n w_n lambda^n grad m^n over the stored adjoint and state planes (trapezoid in
// time), one pass after the backward transport.
template <int DIM>
__global__ __launch_bounds__(BX* BY) void k_body_force(Geo g, const float* __restrict__ lam,
                                                       const float* __restrict__ m,
                                                       float* __restrict__ b) {
  VOXEL_PROLOGUE
  float acc[3] = {0.f, 0.f, 0.f};
  for (int n = 0; n <= g.nt; ++n) {
    const float w = (n == 0 || n == g.nt) ? 0.5f * g.dt : g.dt;
    float gr[3];
    grad_c<DIM>(g, m + (size_t)n * M, x, y, z, p, gr);
    const float wl = w * lam[(size_t)n * M + p];
    for (int c = 0; c < DIM; ++c) acc[c] = fmaf(wl, gr[c], acc[c]);
  }
  for (int c = 0; c < DIM; ++c) b[c * M + p] = acc[c];
}

template <int DIM>
__device__ __forceinline__ float source_f(const Geo& g, const float* __restrict__ m,
                                          const float* __restrict__ dv, int x, int y, int z,
                                          uint32_t p) {
  float gr[3];
  grad_c<DIM>(g, m, x, y, z, p, gr);
  const size_t M = (size_t)g.M;
  float s = gr[0] * dv[p];
  s = fmaf(gr[1], dv[M + p], s);
  if (DIM == 3) s = fmaf(gr[2], dv[2 * M + p], s);
  return -s;
}

template <int DIM>
__global__ __launch_bounds__(BX* BY) void k_inc_init(Geo g, const float* __restrict__ m0,
                                                     const float* __restrict__ dv,
                                                     float* __restrict__ t0) {
  VOXEL_PROLOGUE
  t0[p] = 0.5f * g.dt * source_f<DIM>(g, m0, dv, x, y, z, p);
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* BY) void k_inc_step(Geo g, const float* __restrict__ t_in,
                                                     const float* __restrict__ X,
                                                     const float* __restrict__ m_next,
                                                     const float* __restrict__ dv,
                                                     float* __restrict__ t_out) {
  VOXEL_XY
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    VOXEL_Z(zz)
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    const float tr = apply<DIM>(t_in, make_tap<DIM>(g, x, y, z, ox, oy, oz));
    const float v = fmaf(g.dt, source_f<DIM>(g, m_next, dv, x, y, z, p), tr);
    if (live) t_out[p] = v;
  }
}

template <int DIM>
__global__ __launch_bounds__(BX* BY) void k_inc_last(Geo g, const float* __restrict__ t_in,
                                                     const float* __restrict__ X,
                                                     const float* __restrict__ mT,
                                                     const float* __restrict__ dv,
                                                     float* __restrict__ dlam) {
  VOXEL_PROLOGUE
  const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
  const float tr = apply<DIM>(t_in, make_tap<DIM>(g, x, y, z, ox, oy, oz));
  const float dm = fmaf(0.5f * g.dt, source_f<DIM>(g, mT, dv, x, y, z, p), tr);
  dlam[p] = g.lam_scale * dm;
}

// Deterministic partial sums of (mT - I1)^2: a fixed grid of kRedBlocks blocks, each thread
// a fixed strided subset, then a fixed tree in LDS.
__global__ __launch_bounds__(256) void k_energy_partial(int64_t n, const float* __restrict__ a,
                                                        const float* __restrict__ b,
                                                        double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double d = (double)a[i] - (double)b[i];
    acc = fma(d, d, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

inline dim3 vox_grid(const Geo& g, int zv = 1) {
  return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, (g.nz + zv - 1) / zv);
}
inline dim3 vox_block() { return dim3(BX, BY, 1); }

}  // namespace

#define DISPATCH(KERNEL, ...)                                                       \
  do {                                                                              \
    if (g.dim == 3)                                                                 \
      hipLaunchKernelGGL(KERNEL<3>, vox_grid(g), vox_block(), 0, s, __VA_ARGS__);   \
    else                                                                            \
      hipLaunchKernelGGL(KERNEL<2>, vox_grid(g), vox_block(), 0, s, __VA_ARGS__);   \
  } while (0)

// two voxels per thread along z in 3D, one in 2D
#define DISPATCH_ZV(KERNEL, ...)                                                          \
  do {                                                                                    \
    if (g.dim == 3)                                                                       \
      hipLaunchKernelGGL((KERNEL<3, 2>), vox_grid(g, 2), vox_block(), 0, s, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL((KERNEL<2, 1>), vox_grid(g, 1), vox_block(), 0, s, __VA_ARGS__); \
  } while (0)

void setup(const Geo& g, const float* v, float* X, float* Y, float* a, hipStream_t s) {
  DISPATCH(k_setup, g, v, X, Y, a);
}
void state_step(const Geo& g, const float* m_in, const float* X, float* m_out, hipStream_t s) {
  DISPATCH_ZV(k_state_step, g, m_in, X, m_out);
}
void terminal(const Geo& g, const float* mT, const float* I1, float* lam, hipStream_t s) {
  DISPATCH(k_terminal, g, mT, I1, lam);
}
void adj_step(const Geo& g, const float* lam_in, const float* Y, const float* a, float* lam_out,
              hipStream_t s) {
  DISPATCH_ZV(k_adj_step, g, lam_in, Y, a, lam_out);
}
void body_force(const Geo& g, const float* lam, const float* m, float* b, hipStream_t s) {
  DISPATCH(k_body_force, g, lam, m, b);
}
void inc_init(const Geo& g, const float* m0, const float* dv, float* t0, hipStream_t s) {
  DISPATCH(k_inc_init, g, m0, dv, t0);
}
void inc_step(const Geo& g, const float* t_in, const float* X, const float* m_next,
              const float* dv, float* t_out, hipStream_t s) {
  DISPATCH_ZV(k_inc_step, g, t_in, X, m_next, dv, t_out);
}
void inc_last(const Geo& g, const float* t_in, const float* X, const float* mT,
              const float* dv, float* dlam, hipStream_t s) {
  DISPATCH(k_inc_last, g, t_in, X, mT, dv, dlam);
}
void energy_partial(const Geo& g, const float* mT, const float* I1, double* partial,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_energy_partial, dim3(kRedBlocks), dim3(256), 0, s, g.M, mT, I1, partial);
}

}  // namespace bl
