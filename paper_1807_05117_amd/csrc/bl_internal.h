// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace bl {

// Several problems of one shape in one launch (the batched serving engine).  Problem p's
// device buffers lie p * stride bytes after problem 0's (one arena per problem, equal
// layouts), the launch's gridDim.z is `count` times the single-problem launch's, and the
// blocks of problem p return at once when gate[p * gate_stride] reads 0.  The default (one
// problem, no gate) is the plain launch.  Twiddle tables are read from problem 0 (they depend
// on the grid and band only, which every problem of a batch shares).
struct Batch {
  int64_t stride = 0;
  const int* gate = nullptr;
  int64_t gate_stride = 0;   // ints between consecutive problems' gates
  int count = 1;
};

// problem index of this block, and blockIdx.z within the problem's own launch
__device__ __forceinline__ int batch_pair(const Batch& b) {
  const int zper = b.count > 1 ? (int)gridDim.z / b.count : 0;
  return zper > 0 ? (int)blockIdx.z / zper : 0;
}
__device__ __forceinline__ int batch_bz(const Batch& b, int pair) {
  return (int)blockIdx.z - pair * ((int)gridDim.z / b.count);
}
__device__ __forceinline__ bool batch_gated_off(const Batch& b, int pair) {
  return b.gate != nullptr && b.gate[(size_t)pair * b.gate_stride] == 0;
}
// problem pair's copy of a buffer of problem 0 (null stays null).  Byte-pointer arithmetic,
// not an integer round trip: the compiler then still knows the result points to global memory
// (global and scalar loads; through an integer it can only use flat loads).
template <class T>
__device__ __forceinline__ T* batch_ptr(T* p, const Batch& b, int pair) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p == nullptr ? p : reinterpret_cast<T*>(reinterpret_cast<Byte*>(p) + (int64_t)pair * b.stride);
}
inline dim3 batch_grid(dim3 d, const Batch& b) {
  d.z *= (unsigned)b.count;
  return d;
}
// kernel prologue: the block's problem, gated-off problems return; BL_AT shifts a buffer
#define BL_BATCH(bt)                                  \
  const int bpair_ = ::bl::batch_pair(bt);            \
  if (::bl::batch_gated_off(bt, bpair_)) return;
#define BL_AT(p, bt) p = ::bl::batch_ptr(p, bt, bpair_)

// Sum (MAX: maximum) of one double per thread of a 1D block of 256 threads, in a fixed order:
// within each 64-lane wavefront by shuffles (offsets 32, 16, ..., 1; lane 0 ends with its
// wavefront's value), then the four wavefront values in order by thread 0, which alone returns
// the result.  Every thread of the block must call it (it has two barriers).
template <bool MAX>
__device__ __forceinline__ double block_reduce_256(double v) {
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_down(v, (unsigned)o, 64);
    v = MAX ? fmax(v, w) : v + w;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    r = part[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) r = MAX ? fmax(r, part[w]) : r + part[w];
  }
  __syncthreads();   // part may be reused by a following reduction of the same kernel
  return r;
}

// Kernel timing for the benchmark: a pair of HIP events that the next launch through
// BL_LAUNCH on the calling host thread records at its kernel's own start and end (the
// dispatch's timestamps, no gap to a neighbouring launch).  set_launch_events(e) arms it;
// BL_LAUNCH takes and clears it.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
void set_launch_events(LaunchEvents* e);
LaunchEvents* take_launch_events();
#define BL_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                   \
  do {                                                                                     \
    if (::bl::LaunchEvents* ev_ = ::bl::take_launch_events())                              \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, ev_->start, ev_->stop, 0,  \
                            __VA_ARGS__);                                                  \
    else                                                                                   \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                  \
  } while (0)

// Geometry and weights of one problem, passed by value to every kernel.
struct Geo {
  int dim;            // 2 or 3
  int nx, ny, nz;     // grid (nz == 1 in 2D)
  int kx, ky, kz;     // band (kz == 1 in 2D)
  int kzh;            // stored non-negative kz planes: 1 in 2D, kz/2 in 3D
  int kz0;            // band index of kz = 0: 0 in 2D, kz/2 in 3D
  int nt;             // time steps
  int nref;           // max grid size (voxel size 1/nref)
  int64_t M;          // voxels
  int64_t B;          // band entries per component (kx*ky*kz)
  float dt;           // 1/nt
  float half_nref;    // nref/2 (central difference scale)
  float lam_scale;    // -2/sigma^2
  float inv_nx, inv_ny, inv_nz;   // 1/n per axis (periodic index wrap)
  int gamma;          // 1: incompressible flow (velocities projected divergence-free)
  int newton;         // 1: full Newton Hessian products (else Gauss-Newton)
  int nodes;          // band velocity fields: 1 (stationary) or nt + 1 (one per time node)
  int deform;         // 1: deformation state equation (band displacement of the inverse map)
  int px, py, pz;     // product grid of the truncated convolutions (deformation method)
  // 1: the transports store their outputs with the streaming (non-temporal) hint.  Set when the
  // nine grid fields an incremental step touches exceed the 256 MiB last-level cache: there
  // the hint speeds the steps up, below it the next step's reads of the output would miss.
  int stream_out;
  // launch shapes per kernel class (TR_*): voxels per thread along z of the transports and
  // the setup, the z-chunk multiplier of the iota z stage, the rows per block of the fused
  // iota x/y stage.  Every choice computes bitwise the same values.
  int zv[8];
  // several problems of this shape in one launch (default: one)
  Batch bat;
};

// kernel classes of the launch shapes (Geo::zv)
enum { TR_STATE = 0, TR_INC, TR_ADJ, TR_FORCE, TR_SETUP, TR_IOTA_Z, TR_IOTA_XY, TR_CLASSES };

// Work buffers and twiddle tables of the band<->grid transforms.
constexpr int kYG = 4;     // y outputs per thread in the iota y stage
constexpr int kJG = 8;     // ky outputs per thread in the pi y stage
constexpr int kZP = 64;    // padded row length of the z twiddle table
constexpr int kU = 8;      // loads in flight per thread in the contraction loops
constexpr int kUY = 16;    // loads in flight per thread in the pi y stage

// Twiddle tables are zero-padded so that every chunk of kU loads stays in bounds:
// padded extents: kx, nx rounded up to 8, ny to 32, ky to kJG, nz to 128.
struct DftPlan {
  float2* tw_x = nullptr;   // [kxp][nx]   exp(+2 pi i kx x / nx), kx = j - Kx/2; zero rows >= Kx
  float2* tw_xT = nullptr;  // [nxp][kx]   the same, transposed; zero rows >= nx
  float2* tw_y = nullptr;   // [kyp][nyp]  exp(+2 pi i ky y / ny); zero outside
  float2* tw_yT = nullptr;  // [nyp][kyp]  the same, transposed
  float2* tw_zT = nullptr;  // [nzp][kZP]  exp(+2 pi i h z / nz), h = 0..kzh-1; zero outside
  int kxp = 0, nxp = 0, kyp = 0, nyp = 0, nzp = 0;
  float2* bufA = nullptr;   // stage buffers, each C_max * kzh * max(ky*nx, ny*nx) complex, C_max
                            // the widest transform (4, or every node of a non-stationary field)
  float2* bufB = nullptr;
  // split hi/lo BF16 twiddle matrices of the mixed-precision z stages (FP32 mode: unused)
  unsigned short* wi_bf16 = nullptr;   // [2][nzp32][mixed_kp]    iota: (hi, lo)
  unsigned short* wp_bf16 = nullptr;   // [2][32 mixed_jt][nzp16] pi:   (hi, lo)
  int nzp32 = 0, nzp16 = 0;
  int mixed = 0;
};

constexpr int kMaxKzh = 64;       // register arrays of the z stages: kz <= 128
constexpr int kRedBlocks = 512;   // partial sums per deterministic FP64 reduction

// ---- transforms (bl_dft.hip)
// out: C planes
void iota(const Geo& g, const DftPlan& p, const float2* band, int C, float* out, hipStream_t s);
// pi without the 1/M scale: P[c][h][ky][kx] for h = 0..kzh-1 (half spectrum)
void pi_half(const Geo& g, const DftPlan& p, const float* grid, int C, float2* P, hipStream_t s);
// the stages separately: iota = iota_xy (band -> p.bufB) then iota_z (p.bufB -> out);
// pi_half = pi_z (grid -> p.bufA) then pi_yx (p.bufA -> P)
void iota_xy(const Geo& g, const DftPlan& p, const float2* band, int C, hipStream_t s);
void iota_z(const Geo& g, const DftPlan& p, int C, float* out, hipStream_t s);
void pi_z(const Geo& g, const DftPlan& p, const float* grid, int C, hipStream_t s);
void pi_yx(const Geo& g, const DftPlan& p, int C, float2* P, hipStream_t s);

// ---- mixed-precision z stages on BF16 matrix cores (bl_mixed.hip)
int mixed_kp(const Geo& g);   // padded contraction length of the iota z stage: 2 kzh -> x16
int mixed_jt(const Geo& g);   // 32-row output tiles of the pi z stage
void iota_z_mixed(const Geo& g, const DftPlan& p, const float2* F2, int C, float* out,
                  hipStream_t s);
void pi_z_mixed(const Geo& g, const DftPlan& p, const float* f, int C, float2* G, hipStream_t s);

// ---- band kernels (bl_dft.hip)
// out[c] = projection of raw[c] (c < dim): Hermitian, and divergence-free when g.gamma = 1;
// with_div: out[dim] = spectral divergence.
// reg_partial (may be null): kRedBlocks partial sums of reg_weight * sum_c Lhat |out_c|^2,
// added to the partials already there when reg_accumulate (one velocity per time node).
void band_prep(const Geo& g, const float2* raw, float2* out, int with_div, const double* Lhat64,
               double* reg_partial, hipStream_t s, double reg_weight = 1.0,
               int reg_accumulate = 0);
// the plain projection (no divergence, no regulariser sum) of `nodes` band vectors spaced
// `stride` complex entries apart, in one launch
void band_prep_nodes(const Geo& g, const float2* raw, float2* out, int nodes, size_t stride,
                     hipStream_t s);
// out[c][k] = Lhat(k) vproj[c][k] + scale * P (Hermitian-completed), zero on unpaired planes;
// leray (C == dim): then projected divergence-free per index k.
// With dot_part not NULL (one node), also the finalize_blocks(g) block partials of
// Re sum conj(dotp) out over all C components (each thread sums its band index's components in
// order, then its block in the fixed order of block_reduce_256); with sq_part and max_part not
// NULL likewise the partials of sum |out|^2 and of max |out|.
void band_finalize(const Geo& g, int C, const float2* vproj, const float* Lhat,
                   const float2* P, float scale, float2* out, int* nonfinite, hipStream_t s,
                   int leray = 0, const float2* dotp = nullptr, double* dot_part = nullptr,
                   double* sq_part = nullptr, double* max_part = nullptr);
// blocks of a band_finalize launch (at most kRedBlocks)
int finalize_blocks(const Geo& g);
// band_finalize of `nodes` vectors in one launch: node n reads vproj + n vstride and
// P + n pstride and writes out + n ostride
void band_finalize_nodes(const Geo& g, int C, const float2* vproj, size_t vstride,
                         const float* Lhat, const float2* P, size_t pstride, float scale,
                         float2* out, size_t ostride, int nodes, int* nonfinite, hipStream_t s,
                         int leray = 0);

// ---- transports (bl_transport.hip)
// X: dim planes of forward offsets; YA = (Y, a) backward offsets and reaction factor
void setup(const Geo& g, const float* v, float* X, float4* YA, hipStream_t s);
// non-stationary steps t_n -> t_{n+1} for n < steps, one launch: V holds (v^n, r^n) of every
// node (dim + 1 planes each); step n writes X + n dim M and YA + n M
void setup_ns(const Geo& g, const float* V, float* X, float4* YA, int steps, hipStream_t s);
// b^n = lambda^n grad m^n for the time nodes n < nodes (lam, m: one plane per node; b: dim
// planes per node), one launch; with YA0 (the first step's (Y, a)), lambda^0 is formed from
// lambda^1 as a Interp(lambda^1, i + Y) instead of read (the plane lambda^0 is not used)
void body_nodes(const Geo& g, const float* lam, const float* m, float* b, int nodes,
                hipStream_t s, const float4* YA0 = nullptr);
void state_step(const Geo& g, const float* m_in, const float* X, float* m_out, hipStream_t s);
// kRedBlocks partials of sum (mT - I1)^2 in FP64; with lam not NULL also the terminal adjoint
// lam = lam_scale (mT - I1), the values terminal() writes
void energy_partial(const Geo& g, const float* mT, const float* I1, double* partial,
                    hipStream_t s, float* lam = nullptr);
void terminal(const Geo& g, const float* mT, const float* I1, float* lam, hipStream_t s);
void adj_step(const Geo& g, const float* lam_in, const float4* YA, float* lam_out,
              hipStream_t s);
// b_c = sum_n w_n lam^n d_c m^n over nt + 1 stored planes of lam and m; with YA, lam^0 is
// formed from lam^1 as a Interp(lam^1, i + Y) instead of read (the plane lam^0 is not used)
void body_force(const Geo& g, const float* lam, const float* m, float* b, hipStream_t s,
                const float4* YA = nullptr);
void inc_init(const Geo& g, const float* m0, const float* dv, float* t0, hipStream_t s);
void inc_step(const Geo& g, const float* t_in, const float* X, const float* m_next,
              const float* dv, float* t_out, hipStream_t s);
void inc_last(const Geo& g, const float* t_in, const float* X, const float* mT,
              const float* dv, float* dlam, hipStream_t s);
// full Newton product (the incremental adjoint with its source div(lambda dv), lambda grad dm
// in the body force): incremental state steps that also store dm^{n+1}; the last one also
// forms dlambda^Nt = -(2/sigma^2) dm^Nt + dt/2 div(lambda^Nt dv)
void inc_step_n(const Geo& g, const float* t_in, const float* X, const float* m_next,
                const float* dv, float* t_out, float* dm_out, hipStream_t s);
void inc_last_n(const Geo& g, const float* t_in, const float* X, const float* mT,
                const float* dv, const float* lamT, float* dm_out, float* dlam, hipStream_t s);
// q = a Interp(u_in, i + Y) (+ dt/2 div(lam_n dv) when own); dlam = q; u_out = q + dt/2 div(..)
void adj_step_n(const Geo& g, const float* u_in, const float4* YA, const float* lam_n,
                const float* dv, int own, float* dlam, float* u_out, hipStream_t s);
// b = sum_n w_n (dlam^n grad m^n + lam^n grad dm^n)
void body_force_n(const Geo& g, const float* dlam, const float* m, const float* lam,
                  const float* dm, float* b, hipStream_t s);
// one component of packed float4 voxels into a plane
void unpack4(const Geo& g, int comp, const float4* in, float* plane, hipStream_t s);

// ---- deformation state equation (bl_deform.hip)
// Band fields are full centred bands of g (B entries per component); product-grid planes have
// MP = px * py * pz points; Ph is a kz >= 0 half spectrum of the product grid (pi_half output,
// kzh * ky * kx entries per component) and scaleP = 1 / MP.
// DU[i * dim + j] = d~_j U_i (spectral derivative, lengths of the image grid)
void def_deriv(const Geo& g, const float2* U, float2* DU, hipStream_t s);
// one Runge-Kutta stage st = 1..4 of d_t u~ = -src - conv, conv = Herm(Ph) / MP:
// k = -src - conv; acc = k (st 1), acc + 2k (st 2, 3), acc + k (st 4); the next state
// un + c h k (st 1, 2, 3; c = 1/2, 1/2, 1) or un + h/6 acc (st 4, also stored to unext);
// DU (may be null) receives its spectral derivatives
void def_stage(const Geo& g, float scaleP, const float2* Ph, const float2* src, const float2* un,
               float2* acc, int st, float2* unext, float2* DU, hipStream_t s);
// out_i = sum_j DG[i dim + j] V_j (+ DG2[i dim + j] V2_j when DG2 != null), product grid
void def_prod(const Geo& g, int64_t MP, const float* DG, const float* V, const float* DG2,
              const float* V2, float* out, hipStream_t s);
// kap = h/6 rho, Ksum = kap (start of the transposed sweep)
void def_adj_init(const Geo& g, const float2* rho, float2* kap, float2* Ksum, hipStream_t s);
// KV[i dim + j] = KG_i V_j; GACC_j (+)= sum_i DUG[i dim + j] KG_i (first: =)
void def_adj_prod(const Geo& g, int64_t MP, const float* KG, const float* V, const float* DUG,
                  float* KV, float* GACC, int first, hipStream_t s);
// A_i = sum_j i q_j Herm(Ph[i dim + j]) / MP; the stage st = 4..1 of the transposed sweep
// (next kap, the running sum of A, Ksum += kap; st 1: rho += sum A, then kap = h/6 rho when
// more steps follow)
void def_adj_combine(const Geo& g, float scaleP, const float2* Ph, float2* rho, float2* Asum,
                     float2* Ksum, float2* kap, int st, int more, hipStream_t s);
// out = Lhat vproj (if vproj) + Ksum + Herm(Ph) / MP, divergence-free part when gamma = 1
void def_out(const Geo& g, float scaleP, const float2* Ph, const float2* Ksum,
             const float2* vproj, const float* Lhat, float2* out, int* nonfinite, hipStream_t s);
// image level (image grid): IG = (I0, central-difference gradient of I0)
void def_ig4(const Geo& g, const float* I0, float4* IG, hipStream_t s);
// m1 = I0 and GP = grad I0 interpolated at i + N_ref UG (UG: dim planes, domain units)
void def_warp(const Geo& g, const float* UG, const float4* IG, float* m1, float4* GP,
              hipStream_t s);
// Bf_j = -(2/sigma^2)(m1 - I1) GP_j
void def_rho1(const Geo& g, const float* m1, const float* I1, const float4* GP, float* Bf,
              hipStream_t s);
// Bf_j = -(2/sigma^2) (GP . DU) GP_j with DU = dim planes of iota(du~(1))
void def_drho1(const Geo& g, const float* DU, const float4* GP, float* Bf, hipStream_t s);

// fused stage kernels of the deformation method (bl_deform_fused.hip), 3D product grids with
// pz <= 64 whose tiles fit the LDS budget (fused_ok); F2 and G are work buffers of
// dim^2 * kzh * py * px complex entries (the product plan's bufA / bufB)
bool fused_ok(const Geo& g, const Geo& gp);
// F2[c][h][y][x] from the kz >= 0 half of `in` (dim fields; deriv: the dim^2 fields i q_j in_i)
void fx_iota_xy(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* in, int deriv,
                float2* F2, hipStream_t s);
// columns: iota z, products with VP (+ DUGr . DVP), DUGw <- the derivative fields (if not
// null), pi z of the dim products into G[i][h][y][x]
void fx_col_fwd(const Geo& gp, const DftPlan& pl, const float2* F2, const float* VP,
                float* DUGw, const float* DUGr, const float* DVP, float2* G, hipStream_t s);
// columns: iota z of the cotangent, GACC (+)= (D~U)^T kap, pi z of the dim^2 products kap_i V_j
void fx_col_bwd(const Geo& gp, const DftPlan& pl, const float2* F2, const float* VP,
                const float* DUG, float* GACC, int first, float2* G, hipStream_t s);
// pi xy of G and the Runge-Kutta stage update (as def_stage; wout receives the next state)
void fx_pi_yx_stage(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                    const float2* src, const float2* un, float2* acc, int st, float2* wout,
                    hipStream_t s);
// pi xy of the dim^2 products and the transposed-sweep update (as def_adj_combine)
void fx_pi_yx_adj(const Geo& g, const Geo& gp, const DftPlan& pl, const float2* G, float scaleP,
                  float2* rho, float2* Asum, float2* Ksum, float2* kap, int st, int more,
                  hipStream_t s);

// ---- reductions and band vector algebra (bl_reduce.hip)
// out[0] = sum of n partials in a fixed order (one block); also stored to host[0] (host-mapped
// pinned memory) when host != NULL, and *flag published to host_flag[0] when flag != NULL
void reduce_final(const double* partial, int n, double* out, hipStream_t s,
                  double* host = nullptr, const int* flag = nullptr, double* host_flag = nullptr,
                  const Batch& bt = Batch{});
// kRedBlocks partials of Re sum conj(a) b over n complex entries
void dot_partial(const float2* a, const float2* b, int64_t n, double* partial, hipStream_t s,
                 const Batch& bt = Batch{});
// the same over g.nodes * dim * B entries, node k weighted by the trapezoid weight w_k
void dot_partial_w(const Geo& g, const float2* a, const float2* b, double* partial, hipStream_t s);
// kRedBlocks partials of max |a|
void maxabs_partial(const float2* a, int64_t n, double* partial, hipStream_t s,
                    const Batch& bt = Batch{});
void reduce_max_final(const double* partial, int n, double* out, hipStream_t s,
                      double* host = nullptr, const int* flag = nullptr,
                      double* host_flag = nullptr, const Batch& bt = Batch{});
// reduce_final of pa and, in the same launch, reduce_final (max_b: reduce_max_final) of pb with
// the flag published beside it; the same values as the two separate calls
void reduce_final2(const double* pa, double* outa, double* hosta, const double* pb, double* outb,
                   double* hostb, int n, hipStream_t s, bool max_b = false,
                   const int* flag = nullptr, double* host_flag = nullptr,
                   const Batch& bt = Batch{});
// y = alpha x + y
void axpy(float2* y, const float2* x, double alpha, int64_t n, hipStream_t s,
          const Batch& bt = Batch{});
// host_flag[0] = flag[0] (host-mapped destination)
void publish_flag(const int* flag, double* host_flag, hipStream_t s);
// y = 0; y = x (kernels, so that a captured graph holds no memset or copy node)
void zero_band(float2* y, int64_t n, hipStream_t s, const Batch& bt = Batch{});
void copy_band(float2* y, const float2* x, int64_t n, hipStream_t s, const Batch& bt = Batch{});
// y = x + eps[0] d (step length in device memory)
void add_scaled_dev(float2* y, const float2* x, const float2* d, const double* eps, int64_t n,
                    hipStream_t s, const Batch& bt = Batch{});
// y = x + beta y
void xpby(float2* y, const float2* x, double beta, int64_t n, hipStream_t s);
// one PCG step: pHp = <p, Hp> from its nphp partials php_part (the same value as reduce_final
// of them; stored to pHp[0] and, when not NULL, host-mapped pHp_host[0]),
// alpha = rz / pHp (0 unless pHp > 0), delta += alpha p, r -= alpha Hp, z = r / Lhat,
// kRedBlocks partials of <r, r> (p0) and <r, z> (p1); php_part must not alias p0 or p1
void pcg_step(const Geo& g, const float2* p, const float2* Hp, const double* rz,
              const double* php_part, int nphp, double* pHp, double* pHp_host, float2* delta,
              float2* r, const float* Lhat, float2* z, double* p0, double* p1, hipStream_t s);
// y = x + (num[0] / den[0]) y with device scalars
void xpby_dev(float2* y, const float2* x, const double* num, const double* den, int64_t n,
              hipStream_t s, const Batch& bt = Batch{});
// z = r / Lhat (per component); also kRedBlocks partials of <r, r> (p0) and <r, z> (p1)
void precond_dots(const Geo& g, const float2* r, const float* Lhat, float2* z, double* p0,
                  double* p1, hipStream_t s);
// y = x + eps d
void add_scaled(float2* y, const float2* x, const float2* d, double eps, int64_t n,
                hipStream_t s);
// partials of sum (a - b)^2 over n reals
void sqdiff_partial(const float* a, const float* b, int64_t n, double* partial, hipStream_t s,
                    const Batch& bt = Batch{});

}  // namespace bl
