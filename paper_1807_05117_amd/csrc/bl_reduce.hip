// Deterministic FP64 reductions and band-vector algebra for the Gauss-Newton-Krylov solver
// (paper Section 3.4: PCG on H dv~ = -g~ with preconditioner K~ = L~^-1).
//
// Every reduction runs on a fixed grid of kRedBlocks blocks of 256 threads; each thread
// accumulates a fixed strided subset in FP64, each block reduces its threads' values by
// wavefront shuffles and one fixed-order step across its four wavefronts, and one block sums
// the partials the same way.  No atomics, so results are bitwise repeatable.
#include "bl_internal.h"

namespace bl {
namespace {

// trapezoid weight of the time node of entry i of a stack of g.nodes velocity fields (1 for
// a stationary velocity)
__device__ __forceinline__ double node_weight(const Geo& g, int64_t i) {
  if (g.nodes <= 1) return 1.0;
  const int64_t node = i / ((int64_t)g.dim * g.B);
  const double dt = 1.0 / (double)g.nt;
  return (node == 0 || node == g.nodes - 1) ? 0.5 * dt : dt;
}

__device__ __forceinline__ void block_sum_store(double acc, double* __restrict__ partial) {
  const double r = block_reduce_256<false>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__device__ __forceinline__ void block_max_store(double acc, double* __restrict__ partial) {
  const double r = block_reduce_256<true>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (n); i += (int64_t)gridDim.x * 256)

// Final pass of a reduction: one block sums (or maxes) the partials in a fixed order and
// stores the result in device memory and, when `host` is not NULL, also in host-mapped pinned
// memory, so the host reads it after a stream synchronisation without a separate copy.  With
// `flag` not NULL the non-finite flag of the band kernels is published beside it as a double.
template <bool MAX>
__device__ __forceinline__ void reduce_block(const double* __restrict__ partial, int n,
                                             double* __restrict__ out, double* __restrict__ host,
                                             const int* __restrict__ flag,
                                             double* __restrict__ host_flag) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc = MAX ? fmax(acc, partial[i]) : acc + partial[i];
  const double r = block_reduce_256<MAX>(acc);
  if (threadIdx.x == 0) {
    out[0] = r;
    if (host) host[0] = r;
    if (flag) host_flag[0] = (double)flag[0];
  }
}

template <bool MAX>
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out,
                                                      double* __restrict__ host,
                                                      const int* __restrict__ flag,
                                                      double* __restrict__ host_flag,
                                                      Batch bt) {
  // host-mapped outputs (host, host_flag) belong to single-problem launches only
  BL_BATCH(bt)
  BL_AT(partial, bt);
  BL_AT(out, bt);
  BL_AT(flag, bt);
  reduce_block<MAX>(partial, n, out, host, flag, host_flag);
}

// Two final passes in one launch: block 0 sums the partials pa, block 1 sums (MAXB: takes the
// maximum of) the partials pb and publishes the flag; each exactly as k_reduce_final.
template <bool MAXB>
__global__ __launch_bounds__(256) void k_reduce_final2(const double* __restrict__ pa,
                                                       double* __restrict__ outa,
                                                       double* __restrict__ hosta,
                                                       const double* __restrict__ pb,
                                                       double* __restrict__ outb,
                                                       double* __restrict__ hostb, int n,
                                                       const int* __restrict__ flag,
                                                       double* __restrict__ host_flag, Batch bt) {
  BL_BATCH(bt)
  BL_AT(pa, bt);
  BL_AT(outa, bt);
  BL_AT(pb, bt);
  BL_AT(outb, bt);
  BL_AT(flag, bt);
  if (blockIdx.x == 0)
    reduce_block<false>(pa, n, outa, hosta, nullptr, nullptr);
  else
    reduce_block<MAXB>(pb, n, outb, hostb, flag, host_flag);
}

// One PCG step after the product Hp, in one launch: alpha = rz / pHp (0 unless pHp > 0),
// delta += alpha p, r -= alpha Hp, z = r / Lhat, and the block partials of <r, r> (p0) and
// <r, z> (p1).  Per element the arithmetic of axpy and precond_dots, in the same grid.
__global__ __launch_bounds__(256) void k_pcg_step(Geo g, const float2* __restrict__ p,
                                                  const float2* __restrict__ Hp,
                                                  const double* __restrict__ rz,
                                                  const double* __restrict__ php_part,
                                                  int nphp, double* __restrict__ pHp,
                                                  double* __restrict__ pHp_host,
                                                  float2* __restrict__ delta,
                                                  float2* __restrict__ r,
                                                  const float* __restrict__ Lhat,
                                                  float2* __restrict__ z,
                                                  double* __restrict__ p0,
                                                  double* __restrict__ p1) {
  BL_BATCH(g.bat)
  BL_AT(p, g.bat);
  BL_AT(Hp, g.bat);
  BL_AT(rz, g.bat);
  BL_AT(php_part, g.bat);
  BL_AT(pHp, g.bat);
  BL_AT(delta, g.bat);
  BL_AT(r, g.bat);
  BL_AT(Lhat, g.bat);
  BL_AT(z, g.bat);
  BL_AT(p0, g.bat);
  BL_AT(p1, g.bat);
  const int64_t n = (int64_t)g.nodes * g.dim * g.B;
  // <p, Hp> from its kRedBlocks partials, summed by every block in the order of the final
  // reduction pass; block 0 stores it
  __shared__ double s_php;
  {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nphp; i += 256) acc += php_part[i];
    const double t = block_reduce_256<false>(acc);
    if (threadIdx.x == 0) {
      s_php = t;
      if (blockIdx.x == 0) {
        pHp[0] = t;
        if (pHp_host) pHp_host[0] = t;
      }
    }
    __syncthreads();
  }
  const double d = s_php;
  const double alpha = d > 0.0 ? rz[0] / d : 0.0;
  const double nalpha = d > 0.0 ? -1.0 * (rz[0] / d) : 0.0;
  double rr = 0.0, rzn = 0.0;
  GRID_STRIDE(i, n) {
    const float2 pi = p[i], hi = Hp[i];
    float2 di = delta[i], ri = r[i];
    di.x = (float)fma(alpha, (double)pi.x, (double)di.x);
    di.y = (float)fma(alpha, (double)pi.y, (double)di.y);
    ri.x = (float)fma(nalpha, (double)hi.x, (double)ri.x);
    ri.y = (float)fma(nalpha, (double)hi.y, (double)ri.y);
    delta[i] = di;
    r[i] = ri;
    const int64_t b = i % g.B;
    const float inv = 1.0f / Lhat[b];
    const float2 w = make_float2(ri.x * inv, ri.y * inv);
    z[i] = w;
    if (g.nodes > 1) {
      const double wt = node_weight(g, i);
      rr = fma(wt * (double)ri.x, (double)ri.x, rr);
      rr = fma(wt * (double)ri.y, (double)ri.y, rr);
      rzn = fma(wt * (double)ri.x, (double)w.x, rzn);
      rzn = fma(wt * (double)ri.y, (double)w.y, rzn);
    } else {
      rr = fma((double)ri.x, (double)ri.x, rr);
      rr = fma((double)ri.y, (double)ri.y, rr);
      rzn = fma((double)ri.x, (double)w.x, rzn);
      rzn = fma((double)ri.y, (double)w.y, rzn);
    }
  }
  block_sum_store(rr, p0);
  __syncthreads();
  block_sum_store(rzn, p1);
}

// y = x + (num / den) y: the PCG direction update with beta = <r', z'> / <r, z> on the device
__global__ __launch_bounds__(256) void k_xpby_dev(float2* __restrict__ y, const float2* __restrict__ x,
                                                  const double* __restrict__ num,
                                                  const double* __restrict__ den, int64_t n,
                                                  Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  BL_AT(x, bt);
  BL_AT(num, bt);
  BL_AT(den, bt);
  const double beta = num[0] / den[0];
  GRID_STRIDE(i, n) {
    const float2 a = x[i];
    float2 b = y[i];
    b.x = (float)fma(beta, (double)b.x, (double)a.x);
    b.y = (float)fma(beta, (double)b.y, (double)a.y);
    y[i] = b;
  }
}

__global__ __launch_bounds__(256) void k_dot_partial(const float2* __restrict__ a,
                                                     const float2* __restrict__ b, int64_t n,
                                                     double* __restrict__ partial, Batch bt) {
  BL_BATCH(bt)
  BL_AT(a, bt);
  BL_AT(b, bt);
  BL_AT(partial, bt);
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const float2 x = a[i], y = b[i];
    acc = fma((double)x.x, (double)y.x, acc);
    acc = fma((double)x.y, (double)y.y, acc);
  }
  block_sum_store(acc, partial);
}

__global__ __launch_bounds__(256) void k_dot_partial_w(Geo g, const float2* __restrict__ a,
                                                       const float2* __restrict__ b,
                                                       double* __restrict__ partial) {
  const int64_t n = (int64_t)g.nodes * g.dim * g.B;
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const float2 x = a[i], y = b[i];
    const double wt = node_weight(g, i);
    acc = fma(wt * (double)x.x, (double)y.x, acc);
    acc = fma(wt * (double)x.y, (double)y.y, acc);
  }
  block_sum_store(acc, partial);
}

__global__ __launch_bounds__(256) void k_maxabs_partial(const float2* __restrict__ a, int64_t n,
                                                        double* __restrict__ partial, Batch bt) {
  BL_BATCH(bt)
  BL_AT(a, bt);
  BL_AT(partial, bt);
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const float2 x = a[i];
    acc = fmax(acc, sqrt((double)x.x * x.x + (double)x.y * x.y));
  }
  block_max_store(acc, partial);
}

__global__ __launch_bounds__(256) void k_axpy(float2* __restrict__ y, const float2* __restrict__ x,
                                              double alpha, int64_t n, Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  BL_AT(x, bt);
  GRID_STRIDE(i, n) {
    const float2 a = x[i];
    float2 b = y[i];
    b.x = (float)fma(alpha, (double)a.x, (double)b.x);
    b.y = (float)fma(alpha, (double)a.y, (double)b.y);
    y[i] = b;
  }
}

__global__ __launch_bounds__(256) void k_xpby(float2* __restrict__ y, const float2* __restrict__ x,
                                              double beta, int64_t n) {
  GRID_STRIDE(i, n) {
    const float2 a = x[i];
    float2 b = y[i];
    b.x = (float)fma(beta, (double)b.x, (double)a.x);
    b.y = (float)fma(beta, (double)b.y, (double)a.y);
    y[i] = b;
  }
}

__global__ __launch_bounds__(256) void k_add_scaled(float2* __restrict__ y,
                                                    const float2* __restrict__ x,
                                                    const float2* __restrict__ d, double eps,
                                                    int64_t n, Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  BL_AT(x, bt);
  BL_AT(d, bt);
  GRID_STRIDE(i, n) {
    const float2 a = x[i], b = d[i];
    y[i] = make_float2((float)fma(eps, (double)b.x, (double)a.x),
                       (float)fma(eps, (double)b.y, (double)a.y));
  }
}

__global__ __launch_bounds__(256) void k_precond_dots(Geo g, const float2* __restrict__ r,
                                                      const float* __restrict__ Lhat,
                                                      float2* __restrict__ z,
                                                      double* __restrict__ p0,
                                                      double* __restrict__ p1) {
  BL_BATCH(g.bat)
  BL_AT(r, g.bat);
  BL_AT(Lhat, g.bat);
  BL_AT(z, g.bat);
  BL_AT(p0, g.bat);
  BL_AT(p1, g.bat);
  const int64_t n = (int64_t)g.nodes * g.dim * g.B;
  double rr = 0.0, rz = 0.0;
  GRID_STRIDE(i, n) {
    const int64_t b = i % g.B;
    const float2 x = r[i];
    const float inv = 1.0f / Lhat[b];
    const float2 w = make_float2(x.x * inv, x.y * inv);
    z[i] = w;
    if (g.nodes > 1) {
      const double wt = node_weight(g, i);
      rr = fma(wt * (double)x.x, (double)x.x, rr);
      rr = fma(wt * (double)x.y, (double)x.y, rr);
      rz = fma(wt * (double)x.x, (double)w.x, rz);
      rz = fma(wt * (double)x.y, (double)w.y, rz);
    } else {
      rr = fma((double)x.x, (double)x.x, rr);
      rr = fma((double)x.y, (double)x.y, rr);
      rz = fma((double)x.x, (double)w.x, rz);
      rz = fma((double)x.y, (double)w.y, rz);
    }
  }
  block_sum_store(rr, p0);
  __syncthreads();
  block_sum_store(rz, p1);
}

__global__ __launch_bounds__(256) void k_sqdiff_partial(const float* __restrict__ a,
                                                        const float* __restrict__ b, int64_t n,
                                                        double* __restrict__ partial, Batch bt) {
  BL_BATCH(bt)
  BL_AT(a, bt);
  BL_AT(b, bt);
  BL_AT(partial, bt);
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double d = (double)a[i] - (double)b[i];
    acc = fma(d, d, acc);
  }
  block_sum_store(acc, partial);
}

// y = 0 (a kernel rather than a memset, so that a captured graph holds no memset node)
__global__ __launch_bounds__(256) void k_zero(float2* __restrict__ y, int64_t n, Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  GRID_STRIDE(i, n) y[i] = make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_copy(float2* __restrict__ y, const float2* __restrict__ x,
                                              int64_t n, Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  BL_AT(x, bt);
  GRID_STRIDE(i, n) y[i] = x[i];
}

// y = x + eps d with the step length eps read from device memory
__global__ __launch_bounds__(256) void k_add_scaled_dev(float2* __restrict__ y,
                                                        const float2* __restrict__ x,
                                                        const float2* __restrict__ d,
                                                        const double* __restrict__ epsp,
                                                        int64_t n, Batch bt) {
  BL_BATCH(bt)
  BL_AT(y, bt);
  BL_AT(x, bt);
  BL_AT(d, bt);
  BL_AT(epsp, bt);
  const double eps = epsp[0];
  GRID_STRIDE(i, n) {
    const float2 a = x[i], b = d[i];
    y[i] = make_float2((float)fma(eps, (double)b.x, (double)a.x),
                       (float)fma(eps, (double)b.y, (double)a.y));
  }
}

// the non-finite flag of the band kernels into host-mapped memory (read after one sync)
__global__ void k_publish_flag(const int* __restrict__ flag, double* __restrict__ host_flag) {
  if (threadIdx.x == 0) host_flag[0] = (double)flag[0];
}

inline int blocks_for(int64_t n) {
  (void)n;
  return kRedBlocks;
}

}  // namespace

void reduce_final(const double* partial, int n, double* out, hipStream_t s, double* host,
                  const int* flag, double* host_flag, const Batch& bt) {
  hipLaunchKernelGGL(k_reduce_final<false>, batch_grid(dim3(1), bt), dim3(256), 0, s, partial, n,
                     out, host, flag, host_flag, bt);
}
void reduce_max_final(const double* partial, int n, double* out, hipStream_t s, double* host,
                      const int* flag, double* host_flag, const Batch& bt) {
  hipLaunchKernelGGL(k_reduce_final<true>, batch_grid(dim3(1), bt), dim3(256), 0, s, partial, n,
                     out, host, flag, host_flag, bt);
}
void reduce_final2(const double* pa, double* outa, double* hosta, const double* pb, double* outb,
                   double* hostb, int n, hipStream_t s, bool max_b, const int* flag,
                   double* host_flag, const Batch& bt) {
  if (max_b)
    hipLaunchKernelGGL(k_reduce_final2<true>, batch_grid(dim3(2), bt), dim3(256), 0, s, pa, outa,
                       hosta, pb, outb, hostb, n, flag, host_flag, bt);
  else
    hipLaunchKernelGGL(k_reduce_final2<false>, batch_grid(dim3(2), bt), dim3(256), 0, s, pa, outa,
                       hosta, pb, outb, hostb, n, flag, host_flag, bt);
}
void pcg_step(const Geo& g, const float2* p, const float2* Hp, const double* rz,
              const double* php_part, int nphp, double* pHp, double* pHp_host, float2* delta,
              float2* r, const float* Lhat, float2* z, double* p0, double* p1, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_step, batch_grid(dim3(kRedBlocks), g.bat), dim3(256), 0, s, g, p, Hp,
                     rz, php_part, nphp, pHp, pHp_host, delta, r, Lhat, z, p0, p1);
}
void xpby_dev(float2* y, const float2* x, const double* num, const double* den, int64_t n,
              hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_xpby_dev, batch_grid(dim3(blocks_for(n)), bt), dim3(256), 0, s, y, x, num,
                     den, n, bt);
}
void dot_partial_w(const Geo& g, const float2* a, const float2* b, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial_w, dim3(kRedBlocks), dim3(256), 0, s, g, a, b, partial);
}
void dot_partial(const float2* a, const float2* b, int64_t n, double* partial, hipStream_t s,
                 const Batch& bt) {
  hipLaunchKernelGGL(k_dot_partial, batch_grid(dim3(kRedBlocks), bt), dim3(256), 0, s, a, b, n,
                     partial, bt);
}
void maxabs_partial(const float2* a, int64_t n, double* partial, hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_maxabs_partial, batch_grid(dim3(kRedBlocks), bt), dim3(256), 0, s, a, n,
                     partial, bt);
}
void axpy(float2* y, const float2* x, double alpha, int64_t n, hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_axpy, batch_grid(dim3(blocks_for(n)), bt), dim3(256), 0, s, y, x, alpha, n,
                     bt);
}
void publish_flag(const int* flag, double* host_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_publish_flag, dim3(1), dim3(64), 0, s, flag, host_flag);
}
void zero_band(float2* y, int64_t n, hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_zero, batch_grid(dim3(blocks_for(n)), bt), dim3(256), 0, s, y, n, bt);
}
void copy_band(float2* y, const float2* x, int64_t n, hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_copy, batch_grid(dim3(blocks_for(n)), bt), dim3(256), 0, s, y, x, n, bt);
}
void add_scaled_dev(float2* y, const float2* x, const float2* d, const double* eps, int64_t n,
                    hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_add_scaled_dev, batch_grid(dim3(blocks_for(n)), bt), dim3(256), 0, s, y, x,
                     d, eps, n, bt);
}
void xpby(float2* y, const float2* x, double beta, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_xpby, dim3(blocks_for(n)), dim3(256), 0, s, y, x, beta, n);
}
void add_scaled(float2* y, const float2* x, const float2* d, double eps, int64_t n,
                hipStream_t s) {
  hipLaunchKernelGGL(k_add_scaled, dim3(blocks_for(n)), dim3(256), 0, s, y, x, d, eps, n, Batch{});
}
void precond_dots(const Geo& g, const float2* r, const float* Lhat, float2* z, double* p0,
                  double* p1, hipStream_t s) {
  hipLaunchKernelGGL(k_precond_dots, batch_grid(dim3(kRedBlocks), g.bat), dim3(256), 0, s, g, r,
                     Lhat, z, p0, p1);
}
void sqdiff_partial(const float* a, const float* b, int64_t n, double* partial, hipStream_t s,
                    const Batch& bt) {
  hipLaunchKernelGGL(k_sqdiff_partial, batch_grid(dim3(kRedBlocks), bt), dim3(256), 0, s, a, b, n,
                     partial, bt);
}

}  // namespace bl
