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
// Layout: grid fields are float32 planes with x fastest; vector fields are dim consecutive
// planes.  The backward offsets and the reaction factor are packed into one 16-byte voxel,
// YA = (Y, a), which costs no extra bytes and saves three loads.  The kernels stream at the
// HBM rate, so they read every field once per voxel (12 + 4 + ... bytes) and nothing more;
// the two x-neighbours of every interpolation row come in one 8-byte load.
#include "bl_internal.h"

namespace bl {
namespace {

constexpr int BX = 64;

// Periodic index without branches (|i| < 2^21, so i is exact in float): the quotient from
// i * (1/n) may be off by one near multiples of n, which the two selects correct.  No branch
// keeps the voxels of a thread in one basic block, so their loads can all be in flight.
__device__ __forceinline__ int wrap(int i, int n, float inv_n) {
  const int q = (int)floorf((float)i * inv_n);
  int r = i - q * n;
  r += r < 0 ? n : 0;
  r -= r >= n ? n : 0;
  return r;
}

// Split an offset into the lower cell index (periodic) and the fractional weight.  Offsets
// are clamped to +-2^20 voxels and non-finite offsets are mapped to 0, so every index that
// reaches memory lies in [0, n).
__device__ __forceinline__ void split(float o, int base, int n, float inv_n, int& i0, int& i1,
                                      float& w) {
  if (!(fabsf(o) <= 1048576.0f)) o = 0.0f;
  const float f = floorf(o);
  w = o - f;
  i0 = wrap(base + (int)f, n, inv_n);
  i1 = (i0 + 1 == n) ? 0 : i0 + 1;
}

// Interpolation rows are read through a raw buffer resource: an 8-byte load of two
// consecutive floats needs only 4-byte alignment there (global loads would be split), and the
// hardware range check returns 0 for any dword past the buffer instead of faulting.
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const float* f, const Geo& g) {
  const uint64_t bytes = (uint64_t)g.M * 4u;   // < 2^32: the host limits prod(n) to < 2^30
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(f), (short)0, (int)(uint32_t)bytes,
                                           0x00020000);
}

// f[row + x0] and f[row + x1] where x1 is x0 + 1 or the periodic wrap to 0.  The wrapped
// value comes from a second load that every lane issues; lanes that do not wrap point it past
// the end of the buffer, where the range check returns 0 without touching memory.  No branch.
constexpr uint32_t kPastEnd = 0xFFFFFFFCu;   // >= the byte size of any field (< 2^32)

__device__ __forceinline__ void load_pair(__amdgpu_buffer_rsrc_t rs, uint32_t row, int x0,
                                          int x1, float& v0, float& v1) {
  const f2v v = __builtin_bit_cast(
      f2v, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)((row + (uint32_t)x0) * 4u), 0, 0));
  const bool wrapped = x1 != x0 + 1;
  const uint32_t off = wrapped ? (row + (uint32_t)x1) * 4u : kPastEnd;
  const float w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
  v0 = v.x;
  v1 = wrapped ? w : v.y;
}

// All in-volume indices are 32-bit (the host guarantees prod(n) <= 2^30).
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
  split(ox, x, g.nx, g.inv_nx, t.x0, t.x1, t.wx);
  split(oy, y, g.ny, g.inv_ny, y0, y1, t.wy);
  if (DIM == 3) {
    int z0, z1;
    split(oz, z, g.nz, g.inv_nz, z0, z1, t.wz);
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
__device__ __forceinline__ float apply(__amdgpu_buffer_rsrc_t f, const Tap<DIM>& t) {
  float a0, a1, b0, b1;
  load_pair(f, t.r00, t.x0, t.x1, a0, a1);
  load_pair(f, t.r01, t.x0, t.x1, b0, b1);
  const float ra = fmaf(t.wx, a1 - a0, a0);
  const float rb = fmaf(t.wx, b1 - b0, b0);
  const float pa = fmaf(t.wy, rb - ra, ra);
  if (DIM == 2) return pa;
  float c0, c1, d0, d1;
  load_pair(f, t.r10, t.x0, t.x1, c0, c1);
  load_pair(f, t.r11, t.x0, t.x1, d0, d1);
  const float rc = fmaf(t.wx, c1 - c0, c0);
  const float rd = fmaf(t.wx, d1 - d0, d0);
  const float pb = fmaf(t.wy, rd - rc, rc);
  return fmaf(t.wz, pb - pa, pa);
}

// apply() at the ZV taps of a thread, with the same loaded values and arithmetic, but the
// second loads of wrapped pairs issued only by waves in which some lane wraps (one
// wave-uniform branch after every 8-byte row load of the thread is in flight): waves away
// from the x boundary skip them.  The taps are all formed before the call, so no load of the
// thread waits behind the branch.
template <int DIM, int ZV>
__device__ __forceinline__ void gather_zv(__amdgpu_buffer_rsrc_t f, const Tap<DIM> (&t)[ZV],
                                          float (&out)[ZV]) {
  constexpr int R = DIM == 3 ? 4 : 2;
  f2v v[ZV][R];
  float w[ZV][R];
  bool any = false;
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    const uint32_t rows[4] = {t[zz].r00, t[zz].r01, t[zz].r10, t[zz].r11};
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[zz][r] = __builtin_bit_cast(
          f2v, __builtin_amdgcn_raw_buffer_load_b64(f, (int)((rows[r] + (uint32_t)t[zz].x0) * 4u),
                                                    0, 0));
      w[zz][r] = 0.0f;
    }
    any |= t[zz].x1 != t[zz].x0 + 1;
  }
  if (__builtin_amdgcn_ballot_w64(any) != 0) {
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      const uint32_t rows[4] = {t[zz].r00, t[zz].r01, t[zz].r10, t[zz].r11};
      const bool wrapped = t[zz].x1 != t[zz].x0 + 1;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t off = wrapped ? (rows[r] + (uint32_t)t[zz].x1) * 4u : kPastEnd;
        w[zz][r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(f, (int)off, 0, 0));
      }
    }
  }
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    const bool wrapped = t[zz].x1 != t[zz].x0 + 1;
    float rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float lo = v[zz][r].x, hi = wrapped ? w[zz][r] : v[zz][r].y;
      rr[r] = fmaf(t[zz].wx, hi - lo, lo);
    }
    const float pa = fmaf(t[zz].wy, rr[1] - rr[0], rr[0]);
    if (DIM == 2) {
      out[zz] = pa;
    } else {
      const float pb = fmaf(t[zz].wy, rr[3] - rr[2], rr[2]);
      out[zz] = fmaf(t[zz].wz, pb - pa, pa);
    }
  }
}

// ------------------------------------------------------------------ gather kernels (64 x 4)
// One thread per ZV voxels along z; z is clamped to the grid so that every load stays in
// bounds and the ZV voxels' loads can be issued together; only the stores are guarded.
constexpr int GBY = 4;

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin to the 8
// XCDs, each with its own L2.  The launch is 1D with a multiple of 8 workgroups and workgroup
// b works on tile (b % 8) * (nb / 8) + b / 8 of the x-fastest tile order, so every XCD sweeps
// one contiguous slab of the volume and the y / z neighbours that gathers and central
// differences touch are mostly in its own L2.
constexpr int kXCD = 8;

struct TileIdx {
  int bx, by, bz;
  bool valid;
};

__device__ __forceinline__ TileIdx xcd_tile(int gx, int gy, int gz) {
  const int nb = gridDim.x;                 // multiple of kXCD
  const int b = blockIdx.x;
  const int t = (b % kXCD) * (nb / kXCD) + b / kXCD;
  TileIdx r;
  r.bx = t % gx;
  r.by = (t / gx) % gy;
  r.bz = t / (gx * gy);
  r.valid = r.bz < gz;
  return r;
}

#define GATHER_XY                                                                \
  const TileIdx tile = xcd_tile((g.nx + BX - 1) / BX, (g.ny + GBY - 1) / GBY,    \
                                (g.nz + ZV - 1) / ZV);                           \
  if (!tile.valid) return;                                                       \
  const int x = tile.bx * BX + threadIdx.x;                                      \
  const int y = tile.by * GBY + threadIdx.y;                                     \
  if (x >= g.nx || y >= g.ny) return;
#define GATHER_Z(zz)                                     \
  const int zr = tile.bz * ZV + (zz);                    \
  const int z = zr < g.nz ? zr : g.nz - 1;               \
  const bool live = zr < g.nz;                           \
  const uint32_t p = ((uint32_t)z * g.ny + y) * g.nx + x;
// The values of a thread's ZV voxels are computed first and stored afterwards, so no store
// sits between the voxels' loads.  Large grids store with the streaming hint (Geo::stream_out).
// Both forms are raw buffer stores that differ in their cache-policy immediate (bit 1: nt), so
// the compiler cannot merge the two branches into one plain store.
__device__ __forceinline__ void store_out(const Geo& g, float* out, uint32_t p, float v) {
  const __amdgpu_buffer_rsrc_t rs = field_rsrc(out, g);
  if (g.stream_out)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)(p * 4u), 0, 2);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)(p * 4u), 0, 0);
}
#define STORE_ZV(out, val)                                 \
  _Pragma("unroll") for (int zz = 0; zz < ZV; ++zz) {      \
    GATHER_Z(zz)                                           \
    if (live) store_out(g, (out), p, (val)[zz]);           \
  }

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_setup(Geo g, const float* __restrict__ v,
                                                   float* __restrict__ X,
                                                   float4* __restrict__ YA) {
  BL_BATCH(g.bat)
  BL_AT(v, g.bat);
  BL_AT(X, g.bat);
  BL_AT(YA, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  const float s = g.dt * (float)g.nref;
  // the ZV voxels of the thread are computed first and stored afterwards (their gathers can
  // all be in flight)
  float u[ZV][3];
  Tap<DIM> tf[ZV], tb[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    u[zz][0] = u[zz][1] = u[zz][2] = 0.f;
    for (int c = 0; c < DIM; ++c) u[zz][c] = s * v[c * M + p];
    // forward: X = -(u + Interp(u, i - u)) / 2
    tf[zz] = make_tap<DIM>(g, x, y, z, -u[zz][0], -u[zz][1], -u[zz][2]);
    // backward: Y = +(u + Interp(u, i + u)) / 2
    tb[zz] = make_tap<DIM>(g, x, y, z, u[zz][0], u[zz][1], u[zz][2]);
  }
  float xo[ZV][3], yo[ZV][3], av[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    xo[zz][0] = xo[zz][1] = xo[zz][2] = 0.f;
    yo[zz][0] = yo[zz][1] = yo[zz][2] = 0.f;
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const __amdgpu_buffer_rsrc_t vc = field_rsrc(v + c * M, g);
    float gf[ZV], gb[ZV];
    gather_zv<DIM, ZV>(vc, tf, gf);
    gather_zv<DIM, ZV>(vc, tb, gb);
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      xo[zz][c] = -0.5f * (u[zz][c] + s * gf[zz]);
      yo[zz][c] = 0.5f * (u[zz][c] + s * gb[zz]);
    }
  }
  // reaction factor of the adjoint along the backward characteristic (Heun)
  const float* r = v + DIM * M;
  Tap<DIM> ty[ZV];
  float ri[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    ty[zz] = make_tap<DIM>(g, x, y, z, yo[zz][0], yo[zz][1], yo[zz][2]);
    ri[zz] = r[p];
  }
  float R[ZV];
  gather_zv<DIM, ZV>(field_rsrc(r, g), ty, R);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz)
    av[zz] = 1.0f + 0.5f * g.dt * (R[zz] + (1.0f + g.dt * R[zz]) * ri[zz]);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    if (live) {
      for (int c = 0; c < DIM; ++c) X[c * M + p] = xo[zz][c];
      YA[p] = make_float4(yo[zz][0], yo[zz][1], yo[zz][2], av[zz]);
    }
  }
}

// Non-stationary step t_n -> t_{n+1}: the Heun characteristics take the velocity at both
// ends of the step: X = -(u1 + Interp(u0, i - u1)) / 2 (end point i at t_{n+1}),
// Y = +(u0 + Interp(u1, i + u0)) / 2 (start point i at t_n), R = Interp(r1, i + Y),
// a = 1 + dt/2 [R + (1 + dt R) r0].  With v0 = v1 these are the stationary formulas.
// (every step n of the time grid in one launch: n = blockIdx.y, v0 = V[n], v1 = V[n + 1] with
// dim + 1 planes per node, X[n], YA[n])
template <int DIM>
__global__ __launch_bounds__(BX* GBY) void k_setup_ns(Geo g, const float* __restrict__ V,
                                                      float* __restrict__ Xall,
                                                      float4* __restrict__ YAall) {
  BL_BATCH(g.bat)
  BL_AT(V, g.bat);
  BL_AT(Xall, g.bat);
  BL_AT(YAall, g.bat);
  constexpr int ZV = 1;
  GATHER_XY
  GATHER_Z(0)
  (void)live;
  const size_t M = (size_t)g.M;
  const size_t n = blockIdx.y;
  const float* __restrict__ v0 = V + n * (DIM + 1) * M;
  const float* __restrict__ v1 = v0 + (DIM + 1) * M;
  float* __restrict__ X = Xall + n * DIM * M;
  float4* __restrict__ YA = YAall + n * M;
  const float s = g.dt * (float)g.nref;
  float u0[3] = {0.f, 0.f, 0.f}, u1[3] = {0.f, 0.f, 0.f};
  for (int c = 0; c < DIM; ++c) {
    u0[c] = s * v0[c * M + p];
    u1[c] = s * v1[c * M + p];
  }
  const Tap<DIM> tf[1] = {make_tap<DIM>(g, x, y, z, -u1[0], -u1[1], -u1[2])};
  const Tap<DIM> tb[1] = {make_tap<DIM>(g, x, y, z, u0[0], u0[1], u0[2])};
  float xo[3] = {0.f, 0.f, 0.f}, yo[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    float gf[1], gb[1];
    gather_zv<DIM, 1>(field_rsrc(v0 + c * M, g), tf, gf);
    gather_zv<DIM, 1>(field_rsrc(v1 + c * M, g), tb, gb);
    xo[c] = -0.5f * (u1[c] + s * gf[0]);
    yo[c] = 0.5f * (u0[c] + s * gb[0]);
  }
  const Tap<DIM> ty[1] = {make_tap<DIM>(g, x, y, z, yo[0], yo[1], yo[2])};
  const float ri = v0[DIM * M + p];
  float Rv[1];
  gather_zv<DIM, 1>(field_rsrc(v1 + DIM * M, g), ty, Rv);
  const float R = Rv[0];
  const float a = 1.0f + 0.5f * g.dt * (R + (1.0f + g.dt * R) * ri);
  for (int c = 0; c < DIM; ++c) X[c * M + p] = xo[c];
  YA[p] = make_float4(yo[0], yo[1], yo[2], a);
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_state_step(Geo g, const float* __restrict__ m_in,
                                                        const float* __restrict__ X,
                                                        float* __restrict__ m_out) {
  BL_BATCH(g.bat)
  BL_AT(m_in, g.bat);
  BL_AT(X, g.bat);
  BL_AT(m_out, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  Tap<DIM> tp[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    tp[zz] = make_tap<DIM>(g, x, y, z, ox, oy, oz);
  }
  float val[ZV];
  gather_zv<DIM, ZV>(field_rsrc(m_in, g), tp, val);
  STORE_ZV(m_out, val)
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_adj_step(Geo g, const float* __restrict__ lam_in,
                                                      const float4* __restrict__ YA,
                                                      float* __restrict__ lam_out) {
  BL_BATCH(g.bat)
  BL_AT(lam_in, g.bat);
  BL_AT(YA, g.bat);
  BL_AT(lam_out, g.bat);
  GATHER_XY
  Tap<DIM> tp[ZV];
  float aw[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float4 o = YA[p];
    tp[zz] = make_tap<DIM>(g, x, y, z, o.x, o.y, o.z);
    aw[zz] = o.w;
  }
  float val[ZV];
  gather_zv<DIM, ZV>(field_rsrc(lam_in, g), tp, val);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) val[zz] = aw[zz] * val[zz];
  STORE_ZV(lam_out, val)
}

template <int DIM>
__global__ __launch_bounds__(BX* GBY) void k_terminal(Geo g, const float* __restrict__ mT,
                                                      const float* __restrict__ I1,
                                                      float* __restrict__ lam) {
  BL_BATCH(g.bat)
  BL_AT(mT, g.bat);
  BL_AT(I1, g.bat);
  BL_AT(lam, g.bat);
  constexpr int ZV = 1;
  GATHER_XY
  GATHER_Z(0)
  (void)live;
  lam[p] = g.lam_scale * (mT[p] - I1[p]);
}

// ---------------------------------------------------------------- stencil + gather kernels
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

// f = -grad m . dv at voxel p (dv: dim planes)
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

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_inc_init(Geo g, const float* __restrict__ m0,
                                                      const float* __restrict__ dv,
                                                      float* __restrict__ t0) {
  BL_BATCH(g.bat)
  BL_AT(m0, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(t0, g.bat);
  GATHER_XY
  float val[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    val[zz] = 0.5f * g.dt * source_f<DIM>(g, m0, dv, x, y, z, p);
  }
  STORE_ZV(t0, val)
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_inc_step(Geo g, const float* __restrict__ t_in,
                                                      const float* __restrict__ X,
                                                      const float* __restrict__ m_next,
                                                      const float* __restrict__ dv,
                                                      float* __restrict__ t_out) {
  BL_BATCH(g.bat)
  BL_AT(t_in, g.bat);
  BL_AT(X, g.bat);
  BL_AT(m_next, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(t_out, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  Tap<DIM> tp[ZV];
  float src[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    tp[zz] = make_tap<DIM>(g, x, y, z, ox, oy, oz);
    src[zz] = source_f<DIM>(g, m_next, dv, x, y, z, p);
  }
  float val[ZV];
  gather_zv<DIM, ZV>(field_rsrc(t_in, g), tp, val);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) val[zz] = fmaf(g.dt, src[zz], val[zz]);
  STORE_ZV(t_out, val)
}

template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_inc_last(Geo g, const float* __restrict__ t_in,
                                                      const float* __restrict__ X,
                                                      const float* __restrict__ mT,
                                                      const float* __restrict__ dv,
                                                      float* __restrict__ dlam) {
  BL_BATCH(g.bat)
  BL_AT(t_in, g.bat);
  BL_AT(X, g.bat);
  BL_AT(mT, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(dlam, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  Tap<DIM> tp[ZV];
  float src[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    tp[zz] = make_tap<DIM>(g, x, y, z, ox, oy, oz);
    src[zz] = source_f<DIM>(g, mT, dv, x, y, z, p);
  }
  float val[ZV];
  gather_zv<DIM, ZV>(field_rsrc(t_in, g), tp, val);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) val[zz] = g.lam_scale * fmaf(0.5f * g.dt, src[zz], val[zz]);
  STORE_ZV(dlam, val)
}

// b = sum_n w_n lambda^n grad m^n over the stored adjoint and state planes (trapezoid in
// time), one pass after the backward transport.  A thread takes its ZV voxels of a z run for
// every time node in turn (node loop outside, voxel loop inside), so its z differences come
// from a sliding window of three planes held in registers: each m^n plane of the run is read
// once, plus one plane above and below, and the ZV voxels' loads of a node are in flight
// together.  With YA given, lambda^0 is not read: it is formed here as the last adjoint step
// would, a Interp(lambda^1, i + Y), with the same arithmetic (the caller then stops the
// backward transport at lambda^1; lambda^0 is needed by nothing but this sum).
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_body_force(Geo g, const float* __restrict__ lam,
                                                        const float* __restrict__ m,
                                                        float* __restrict__ b,
                                                        const float4* __restrict__ YA) {
  BL_BATCH(g.bat)
  BL_AT(lam, g.bat);
  BL_AT(m, g.bat);
  BL_AT(b, g.bat);
  BL_AT(YA, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  const uint32_t sz = (uint32_t)g.nx * g.ny;
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
  const uint32_t sy = g.nx;
  float acc[ZV][3];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) acc[zz][0] = acc[zz][1] = acc[zz][2] = 0.f;
  // the run's first voxel and its lower z neighbour (periodic); the run starts below nz
  const int z0 = tile.bz * ZV;
  const uint32_t p0 = ((uint32_t)z0 * g.ny + y) * g.nx + x;
  const uint32_t p0m = z0 == 0 ? p0 + (uint32_t)(g.nz - 1) * sz : p0 - sz;
  // lambda^0 of the thread's voxels from lambda^1 (as k_adj_step)
  float l0[ZV];
  const bool form0 = YA != nullptr;
  if (form0) {
    Tap<DIM> tp[ZV];
    float aw[ZV];
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      GATHER_Z(zz)
      (void)live;
      const float4 o = YA[p];
      tp[zz] = make_tap<DIM>(g, x, y, z, o.x, o.y, o.z);
      aw[zz] = o.w;
    }
    gather_zv<DIM, ZV>(field_rsrc(lam + M, g), tp, l0);
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) l0[zz] = aw[zz] * l0[zz];
  }
  // one time node: own = lambda^n from l0 (n = 0 only), else from its stored plane
  auto node = [&](int n, bool own) {
    const float w = (n == 0 || n == g.nt) ? 0.5f * g.dt : g.dt;
    const float* __restrict__ mn = m + n * M;
    const float* __restrict__ ln = lam + n * M;
    float prev = DIM == 3 ? mn[p0m] : 0.f;   // m at z - 1
    float cur = DIM == 3 ? mn[p0] : 0.f;     // m at z
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      GATHER_Z(zz)
      (void)live;
      const uint32_t row = p - x;
      const float gx = (mn[row + xp] - mn[row + xm]) * g.half_nref;
      const uint32_t pym = y == 0 ? p + (uint32_t)(g.ny - 1) * sy : p - sy;
      const uint32_t pyp = y + 1 == g.ny ? p - (uint32_t)(g.ny - 1) * sy : p + sy;
      const float gy = (mn[pyp] - mn[pym]) * g.half_nref;
      float gz = 0.f;
      if (DIM == 3) {
        // voxels past nz repeat the clamped last plane and are not stored
        const uint32_t pzp = z + 1 == g.nz ? p - (uint32_t)(g.nz - 1) * sz : p + sz;
        const float next = mn[pzp];
        gz = (next - prev) * g.half_nref;
        prev = cur;
        cur = next;
      }
      const float wl = w * (own ? l0[zz] : ln[p]);
      acc[zz][0] = fmaf(wl, gx, acc[zz][0]);
      acc[zz][1] = fmaf(wl, gy, acc[zz][1]);
      if (DIM == 3) acc[zz][2] = fmaf(wl, gz, acc[zz][2]);
    }
  };
  if (form0) node(0, true);
  else node(0, false);
  for (int n = 1; n <= g.nt; ++n) node(n, false);
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    if (live)
      for (int c = 0; c < DIM; ++c) b[c * M + p] = acc[zz][c];
  }
}

// ------------------------------------------------------------ full Newton Hessian product
// The Newton product keeps the adjoint terms the Gauss-Newton one drops: the source
// s^n = div(lambda^n dv) of the incremental adjoint and lambda^n grad dm^n in the body force.
// The incremental state steps also store dm^n; the incremental adjoint runs on
//   q^Nt = -(2/sigma^2) dm^Nt,  dlambda^Nt = u^Nt = q^Nt + dt/2 s^Nt,
//   q^n = a Interp(u^{n+1}, i + Y) + dt/2 s^n,  dlambda^n = q^n,  u^n = q^n + dt/2 s^n  (0 < n < Nt),
//   dlambda^0 = a Interp(u^1, i + Y).

// central-difference divergence of lambda dv at voxel p: sum_j (lam dv_j)(i + e_j) - (i - e_j)
template <int DIM>
__device__ __forceinline__ float div_lam_dv(const Geo& g, const float* __restrict__ lam,
                                            const float* __restrict__ dv, int x, int y, int z,
                                            uint32_t p) {
  const size_t M = (size_t)g.M;
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
  const uint32_t row = p - x;
  float s = lam[row + xp] * dv[row + xp] - lam[row + xm] * dv[row + xm];
  const uint32_t sy = g.nx;
  const uint32_t pym = y == 0 ? p + (uint32_t)(g.ny - 1) * sy : p - sy;
  const uint32_t pyp = y + 1 == g.ny ? p - (uint32_t)(g.ny - 1) * sy : p + sy;
  s += lam[pyp] * dv[M + pyp] - lam[pym] * dv[M + pym];
  if (DIM == 3) {
    const uint32_t sz = (uint32_t)g.nx * g.ny;
    const uint32_t pzm = z == 0 ? p + (uint32_t)(g.nz - 1) * sz : p - sz;
    const uint32_t pzp = z + 1 == g.nz ? p - (uint32_t)(g.nz - 1) * sz : p + sz;
    s += lam[pzp] * dv[2 * M + pzp] - lam[pzm] * dv[2 * M + pzm];
  }
  return s * g.half_nref;
}

// incremental state step that also stores dm^{n+1} = Interp(t^n, i + X) + dt/2 f^{n+1}
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_inc_step_n(Geo g, const float* __restrict__ t_in,
                                                        const float* __restrict__ X,
                                                        const float* __restrict__ m_next,
                                                        const float* __restrict__ dv,
                                                        float* __restrict__ t_out,
                                                        float* __restrict__ dm_out) {
  BL_BATCH(g.bat)
  BL_AT(t_in, g.bat);
  BL_AT(X, g.bat);
  BL_AT(m_next, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(t_out, g.bat);
  BL_AT(dm_out, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  float val[ZV], dmv[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    const float tr = apply<DIM>(field_rsrc(t_in, g), make_tap<DIM>(g, x, y, z, ox, oy, oz));
    const float f = source_f<DIM>(g, m_next, dv, x, y, z, p);
    val[zz] = fmaf(g.dt, f, tr);
    dmv[zz] = fmaf(0.5f * g.dt, f, tr);
  }
  STORE_ZV(t_out, val)
  STORE_ZV(dm_out, dmv)
}

// last incremental state step: dm^Nt, and dlambda^Nt = u^Nt = -(2/sigma^2) dm^Nt + dt/2 s^Nt
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_inc_last_n(Geo g, const float* __restrict__ t_in,
                                                        const float* __restrict__ X,
                                                        const float* __restrict__ mT,
                                                        const float* __restrict__ dv,
                                                        const float* __restrict__ lamT,
                                                        float* __restrict__ dm_out,
                                                        float* __restrict__ dlam) {
  BL_BATCH(g.bat)
  BL_AT(t_in, g.bat);
  BL_AT(X, g.bat);
  BL_AT(mT, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(lamT, g.bat);
  BL_AT(dm_out, g.bat);
  BL_AT(dlam, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  float dmv[ZV], val[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float ox = X[p], oy = X[M + p], oz = DIM == 3 ? X[2 * M + p] : 0.f;
    const float tr = apply<DIM>(field_rsrc(t_in, g), make_tap<DIM>(g, x, y, z, ox, oy, oz));
    const float dm = fmaf(0.5f * g.dt, source_f<DIM>(g, mT, dv, x, y, z, p), tr);
    dmv[zz] = dm;
    val[zz] = fmaf(0.5f * g.dt, div_lam_dv<DIM>(g, lamT, dv, x, y, z, p), g.lam_scale * dm);
  }
  STORE_ZV(dm_out, dmv)
  STORE_ZV(dlam, val)
}

// one incremental adjoint step of the Newton product: q = a Interp(u^{n+1}, i + Y) (+ dt/2 s^n
// when own); dlambda^n = q; with u_out, u^n = q + dt/2 s^n
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_adj_step_n(Geo g, const float* __restrict__ u_in,
                                                        const float4* __restrict__ YA,
                                                        const float* __restrict__ lam_n,
                                                        const float* __restrict__ dv, int own,
                                                        float* __restrict__ dlam,
                                                        float* __restrict__ u_out) {
  BL_BATCH(g.bat)
  BL_AT(u_in, g.bat);
  BL_AT(YA, g.bat);
  BL_AT(lam_n, g.bat);
  BL_AT(dv, g.bat);
  BL_AT(dlam, g.bat);
  BL_AT(u_out, g.bat);
  GATHER_XY
  float qv[ZV], uv[ZV];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    const float4 o = YA[p];
    const float tr = o.w * apply<DIM>(field_rsrc(u_in, g), make_tap<DIM>(g, x, y, z, o.x, o.y, o.z));
    const float hs = own ? 0.5f * g.dt * div_lam_dv<DIM>(g, lam_n, dv, x, y, z, p) : 0.f;
    qv[zz] = tr + hs;
    uv[zz] = qv[zz] + hs;
  }
  STORE_ZV(dlam, qv)
  if (u_out) { STORE_ZV(u_out, uv) }
}

// Newton body force: sum_n w_n (dlambda^n grad m^n + lambda^n grad dm^n); the node loop is
// outside the thread's z run and the z differences of m^n and dm^n come from sliding windows,
// as in k_body_force
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_body_force_n(Geo g, const float* __restrict__ dlam,
                                                          const float* __restrict__ m,
                                                          const float* __restrict__ lam,
                                                          const float* __restrict__ dm,
                                                          float* __restrict__ b) {
  BL_BATCH(g.bat)
  BL_AT(dlam, g.bat);
  BL_AT(m, g.bat);
  BL_AT(lam, g.bat);
  BL_AT(dm, g.bat);
  BL_AT(b, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  const uint32_t sz = (uint32_t)g.nx * g.ny;
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
  const uint32_t sy = g.nx;
  float acc[ZV][3];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) acc[zz][0] = acc[zz][1] = acc[zz][2] = 0.f;
  const int z0 = tile.bz * ZV;
  const uint32_t p0 = ((uint32_t)z0 * g.ny + y) * g.nx + x;
  const uint32_t p0m = z0 == 0 ? p0 + (uint32_t)(g.nz - 1) * sz : p0 - sz;
  for (int n = 0; n <= g.nt; ++n) {
    const float w = (n == 0 || n == g.nt) ? 0.5f * g.dt : g.dt;
    const float* __restrict__ mn = m + n * M;
    const float* __restrict__ dn = dm + n * M;
    float mprev = DIM == 3 ? mn[p0m] : 0.f, mcur = DIM == 3 ? mn[p0] : 0.f;
    float dprev = DIM == 3 ? dn[p0m] : 0.f, dcur = DIM == 3 ? dn[p0] : 0.f;
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      GATHER_Z(zz)
      (void)live;
      const uint32_t row = p - x;
      const uint32_t pym = y == 0 ? p + (uint32_t)(g.ny - 1) * sy : p - sy;
      const uint32_t pyp = y + 1 == g.ny ? p - (uint32_t)(g.ny - 1) * sy : p + sy;
      float gr[3], gd[3];
      gr[0] = (mn[row + xp] - mn[row + xm]) * g.half_nref;
      gr[1] = (mn[pyp] - mn[pym]) * g.half_nref;
      gd[0] = (dn[row + xp] - dn[row + xm]) * g.half_nref;
      gd[1] = (dn[pyp] - dn[pym]) * g.half_nref;
      gr[2] = gd[2] = 0.f;
      if (DIM == 3) {
        const uint32_t pzp = z + 1 == g.nz ? p - (uint32_t)(g.nz - 1) * sz : p + sz;
        const float mnext = mn[pzp], dnext = dn[pzp];
        gr[2] = (mnext - mprev) * g.half_nref;
        gd[2] = (dnext - dprev) * g.half_nref;
        mprev = mcur;
        mcur = mnext;
        dprev = dcur;
        dcur = dnext;
      }
      const float wl = w * dlam[n * M + p];
      const float wa = w * lam[n * M + p];
#pragma unroll
      for (int c = 0; c < DIM; ++c) acc[zz][c] = fmaf(wa, gd[c], fmaf(wl, gr[c], acc[zz][c]));
    }
  }
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    if (live)
      for (int c = 0; c < DIM; ++c) b[c * M + p] = acc[zz][c];
  }
}

// b^n = lambda^n grad m^n at the time node n = blockIdx.y (a non-stationary gradient or
// product has one body force per node, not a time integral); all nodes in one launch
template <int DIM, int ZV>
__global__ __launch_bounds__(BX* GBY) void k_body_node(Geo g, const float* __restrict__ lam,
                                                       const float* __restrict__ m,
                                                       float* __restrict__ b,
                                                       const float4* __restrict__ YA0) {
  BL_BATCH(g.bat)
  BL_AT(lam, g.bat);
  BL_AT(m, g.bat);
  BL_AT(b, g.bat);
  BL_AT(YA0, g.bat);
  GATHER_XY
  const size_t M = (size_t)g.M;
  // with YA0 (the first step's (Y, a)), the blocks of node 0 form lambda^0 = a Interp(lambda^1,
  // i + Y) as the adjoint step would, with the same arithmetic, instead of reading it
  const bool form0 = YA0 != nullptr && blockIdx.y == 0;
  float l0[ZV];
  if (form0) {
    Tap<DIM> tp[ZV];
    float aw[ZV];
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) {
      GATHER_Z(zz)
      (void)live;
      const float4 o = YA0[p];
      tp[zz] = make_tap<DIM>(g, x, y, z, o.x, o.y, o.z);
      aw[zz] = o.w;
    }
    gather_zv<DIM, ZV>(field_rsrc(lam + M, g), tp, l0);
#pragma unroll
    for (int zz = 0; zz < ZV; ++zz) l0[zz] = aw[zz] * l0[zz];
  }
  lam += blockIdx.y * M;
  m += blockIdx.y * M;
  b += blockIdx.y * (size_t)DIM * M;
  float acc[ZV][3];
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    (void)live;
    float gr[3];
    grad_c<DIM>(g, m, x, y, z, p, gr);
    const float l = form0 ? l0[zz] : lam[p];
    for (int c = 0; c < DIM; ++c) acc[zz][c] = l * gr[c];
  }
#pragma unroll
  for (int zz = 0; zz < ZV; ++zz) {
    GATHER_Z(zz)
    if (live)
      for (int c = 0; c < DIM; ++c) b[c * M + p] = acc[zz][c];
  }
}

// Deterministic partial sums of (mT - I1)^2: a fixed grid of kRedBlocks blocks, each thread
// a fixed strided subset, then the fixed-order block reduction (wavefront shuffles).
__global__ __launch_bounds__(256) void k_energy_partial(int64_t n, const float* __restrict__ a,
                                                        const float* __restrict__ b,
                                                        double* __restrict__ partial,
                                                        float* __restrict__ lam, float lam_scale,
                                                        Batch bt) {
  BL_BATCH(bt)
  BL_AT(a, bt);
  BL_AT(b, bt);
  BL_AT(partial, bt);
  BL_AT(lam, bt);
  // the thread's elements i, i + stride, ... in that order; kEU of them per round with all of
  // the round's loads issued before its stores (a loop that loads and stores one element per
  // iteration waits for each iteration's loads)
  constexpr int kEU = 8;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  for (; i + (kEU - 1) * stride < n; i += kEU * stride) {
    float av[kEU], bv[kEU];
#pragma unroll
    for (int u = 0; u < kEU; ++u) {
      av[u] = a[i + u * stride];
      bv[u] = b[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < kEU; ++u) {
      const double d = (double)av[u] - (double)bv[u];
      acc = fma(d, d, acc);
      if (lam) lam[i + u * stride] = lam_scale * (av[u] - bv[u]);   // as k_terminal forms it
    }
  }
  for (; i < n; i += stride) {
    const float ai = a[i], bi = b[i];
    const double d = (double)ai - (double)bi;
    acc = fma(d, d, acc);
    if (lam) lam[i] = lam_scale * (ai - bi);
  }
  const double r = block_reduce_256<false>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// One component of packed float4 data into a plane.
__global__ __launch_bounds__(256) void k_unpack4(int64_t n, int comp,
                                                 const float4* __restrict__ src,
                                                 float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4 v = src[i];
  dst[i] = comp == 0 ? v.x : comp == 1 ? v.y : comp == 2 ? v.z : v.w;
}

inline dim3 gather_grid(const Geo& g, int zv) {
  const long long nb = (long long)((g.nx + BX - 1) / BX) * ((g.ny + GBY - 1) / GBY) *
                       ((g.nz + zv - 1) / zv);
  return dim3((unsigned)((nb + kXCD - 1) / kXCD * kXCD));
}
}  // namespace

// 3D launches take the class's voxels per thread along z (1, 2, 4 or 8); 2D runs one per thread.
// NY > 1 repeats the grid over blockIdx.y (one copy per time node).
#define GRID_N(ZV_, NY) batch_grid(dim3(gather_grid(g, ZV_).x, (NY)), g.bat)
#define DISPATCH_GATHER_N(KERNEL, CLS, NY, ...)                                                 \
  do {                                                                                          \
    if (g.dim == 3) {                                                                           \
      const int zv_ = g.zv[CLS];                                                                \
      if (zv_ == 8)                                                                             \
        BL_LAUNCH((KERNEL<3, 8>), GRID_N(8, NY), dim3(BX, GBY), 0, s, __VA_ARGS__);    \
      else if (zv_ == 4)                                                                        \
        BL_LAUNCH((KERNEL<3, 4>), GRID_N(4, NY), dim3(BX, GBY), 0, s, __VA_ARGS__);    \
      else if (zv_ == 2)                                                                        \
        BL_LAUNCH((KERNEL<3, 2>), GRID_N(2, NY), dim3(BX, GBY), 0, s, __VA_ARGS__);    \
      else                                                                                      \
        BL_LAUNCH((KERNEL<3, 1>), GRID_N(1, NY), dim3(BX, GBY), 0, s, __VA_ARGS__);    \
    } else {                                                                                    \
      BL_LAUNCH((KERNEL<2, 1>), GRID_N(1, NY), dim3(BX, GBY), 0, s, __VA_ARGS__);     \
    }                                                                                           \
  } while (0)
#define DISPATCH_GATHER(KERNEL, CLS, ...) DISPATCH_GATHER_N(KERNEL, CLS, 1, __VA_ARGS__)
#define DISPATCH_ONE(KERNEL, ...)                                                          \
  do {                                                                                     \
    if (g.dim == 3)                                                                        \
      hipLaunchKernelGGL(KERNEL<3>, batch_grid(gather_grid(g, 1), g.bat), dim3(BX, GBY), 0, s, \
                         __VA_ARGS__);                                                     \
    else                                                                                   \
      hipLaunchKernelGGL(KERNEL<2>, batch_grid(gather_grid(g, 1), g.bat), dim3(BX, GBY), 0, s, \
                         __VA_ARGS__);                                                     \
  } while (0)
void setup(const Geo& g, const float* v, float* X, float4* YA, hipStream_t s) {
  DISPATCH_GATHER(k_setup, TR_SETUP, g, v, X, YA);
}
void setup_ns(const Geo& g, const float* V, float* X, float4* YA, int steps, hipStream_t s) {
  const dim3 grid = batch_grid(dim3(gather_grid(g, 1).x, (unsigned)steps), g.bat);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_setup_ns<3>, grid, dim3(BX, GBY), 0, s, g, V, X, YA);
  else
    hipLaunchKernelGGL(k_setup_ns<2>, grid, dim3(BX, GBY), 0, s, g, V, X, YA);
}
void body_nodes(const Geo& g, const float* lam, const float* m, float* b, int nodes,
                hipStream_t s, const float4* YA0) {
  DISPATCH_GATHER_N(k_body_node, TR_FORCE, nodes, g, lam, m, b, YA0);
}
void state_step(const Geo& g, const float* m_in, const float* X, float* m_out, hipStream_t s) {
  DISPATCH_GATHER(k_state_step, TR_STATE, g, m_in, X, m_out);
}
void terminal(const Geo& g, const float* mT, const float* I1, float* lam, hipStream_t s) {
  DISPATCH_ONE(k_terminal, g, mT, I1, lam);
}
void adj_step(const Geo& g, const float* lam_in, const float4* YA, float* lam_out,
              hipStream_t s) {
  DISPATCH_GATHER(k_adj_step, TR_ADJ, g, lam_in, YA, lam_out);
}
void body_force(const Geo& g, const float* lam, const float* m, float* b, hipStream_t s,
                const float4* YA) {
  DISPATCH_GATHER(k_body_force, TR_FORCE, g, lam, m, b, YA);
}
void inc_init(const Geo& g, const float* m0, const float* dv, float* t0, hipStream_t s) {
  DISPATCH_GATHER(k_inc_init, TR_INC, g, m0, dv, t0);
}
void inc_step(const Geo& g, const float* t_in, const float* X, const float* m_next,
              const float* dv, float* t_out, hipStream_t s) {
  DISPATCH_GATHER(k_inc_step, TR_INC, g, t_in, X, m_next, dv, t_out);
}
void inc_last(const Geo& g, const float* t_in, const float* X, const float* mT,
              const float* dv, float* dlam, hipStream_t s) {
  DISPATCH_GATHER(k_inc_last, TR_INC, g, t_in, X, mT, dv, dlam);
}
void inc_step_n(const Geo& g, const float* t_in, const float* X, const float* m_next,
                const float* dv, float* t_out, float* dm_out, hipStream_t s) {
  DISPATCH_GATHER(k_inc_step_n, TR_INC, g, t_in, X, m_next, dv, t_out, dm_out);
}
void inc_last_n(const Geo& g, const float* t_in, const float* X, const float* mT,
                const float* dv, const float* lamT, float* dm_out, float* dlam, hipStream_t s) {
  DISPATCH_GATHER(k_inc_last_n, TR_INC, g, t_in, X, mT, dv, lamT, dm_out, dlam);
}
void adj_step_n(const Geo& g, const float* u_in, const float4* YA, const float* lam_n,
                const float* dv, int own, float* dlam, float* u_out, hipStream_t s) {
  DISPATCH_GATHER(k_adj_step_n, TR_ADJ, g, u_in, YA, lam_n, dv, own, dlam, u_out);
}
void body_force_n(const Geo& g, const float* dlam, const float* m, const float* lam,
                  const float* dm, float* b, hipStream_t s) {
  DISPATCH_GATHER(k_body_force_n, TR_FORCE, g, dlam, m, lam, dm, b);
}
void energy_partial(const Geo& g, const float* mT, const float* I1, double* partial,
                    hipStream_t s, float* lam) {
  hipLaunchKernelGGL(k_energy_partial, batch_grid(dim3(kRedBlocks), g.bat), dim3(256), 0, s, g.M,
                     mT, I1, partial, lam, g.lam_scale, g.bat);
}
void unpack4(const Geo& g, int comp, const float4* in, float* plane, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack4, dim3((unsigned)((g.M + 255) / 256)), dim3(256), 0, s, g.M, comp,
                     in, plane);
}

}  // namespace bl
