// Internal declarations of the sscg library: device data layouts, job tables for
// grouped kernel launches, solver state and the launcher functions each .hip file
// provides. Not part of the public ABI (include/sscg.h is).
//
// Internal spinor layout ("planar"): [source][12 components][V sites], one complex
// number (double2 / float2) per entry, component c = 3 spin + colour. A thread
// that owns site s touches entry c*V + s of every plane, so a wavefront reads
// 64 consecutive complex numbers per plane (coalesced).
// Internal gauge layout: [4 mu][LR/2 entries][V], entry e = 3 row + col of
// U_mu(s); with LR = 12 only rows 0 and 1 are stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>
#include <vector>

namespace sscg {

constexpr int kMaxJobs = 8;   // problems in one grouped launch
constexpr int kBlock = 256;   // threads per block for streaming kernels

template <typename T> struct V2t;
template <> struct V2t<double> { using type = double2; };
template <> struct V2t<float> { using type = float2; };
template <typename T> using V2 = typename V2t<T>::type;

// ---- complex helpers on double2 / float2 -----------------------------------
template <typename C> __host__ __device__ __forceinline__ C cmk(decltype(C{}.x) re, decltype(C{}.x) im) { C c; c.x = re; c.y = im; return c; }
__host__ __device__ __forceinline__ double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
  C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
// conj(a) * b
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
  C c; c.x = a.x * b.x + a.y * b.y; c.y = a.x * b.y - a.y * b.x; return c;
}
// acc += a * b
// (written as chains of fused multiply-adds: four per complex product)
template <typename C> __host__ __device__ __forceinline__ void cfma(C &acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename C> __host__ __device__ __forceinline__ void cfmac(C &acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
template <typename C> __host__ __device__ __forceinline__ C cscale(C a, decltype(C{}.x) s) { C c; c.x = a.x * s; c.y = a.y * s; return c; }
// i * a
template <typename C> __host__ __device__ __forceinline__ C ci(C a) { C c; c.x = -a.y; c.y = a.x; return c; }
// -i * a
template <typename C> __host__ __device__ __forceinline__ C cmi(C a) { C c; c.x = a.y; c.y = -a.x; return c; }
template <typename C> __host__ __device__ __forceinline__ C cneg(C a) { C c; c.x = -a.x; c.y = -a.y; return c; }

// ---- solver state (device memory) ------------------------------------------
// Per source: the seed CG scalars of (sigma I - A) x = v.
struct SeedState {
  double rho;        // <r_k, r_k>
  double alpha;      // alpha_k of the current iteration
  double alpha_prev; // alpha_{k-1} (1 before the first iteration)
  double beta_prev;  // beta_{k-1} (0 before the first iteration)
  double vnorm;      // ||v||
  double maxres;     // max over active shifts of ||r_j|| / ||v|| after the last update
  int32_t iters;     // completed iterations
  int32_t done;      // 1: no more work for this source
  int32_t status;    // SSCG_OK / SSCG_ENOTCONV / SSCG_EBREAKDOWN
  int32_t nactive;   // shifts still iterating
  int32_t pending;   // 1: shift update of the current iteration still to apply
  int32_t pad;
};
// Per (source, shift): the scalars of shift j (s_j = z_j - sigma).
struct ShiftState {
  double2 s;
  double2 pi_prev, pi_cur;   // pi_{j,k-1}, pi_{j,k}
  double2 a, b, ipi;         // alpha_{j,k}, beta_{j,k}, 1/pi_{j,k+1}
  int32_t active;            // still iterating (before this iteration's decision)
  int32_t upd;               // apply the update of the current iteration
  int32_t conv_iter;         // iteration after which it froze, -1 if not yet
  int32_t pad;
  double tscale;             // this shift's tolerance multiplier (1: the common tol)
  double pad2;
};

// ---- job tables -------------------------------------------------------------
// A grouped launch covers up to kMaxJobs problems; block b belongs to the job
// whose [block_begin, block_begin + nblocks) range contains it.
struct DslashJob {
  const void *in;        // planar [nsrc][12][V] of T
  void *out;             // planar [nsrc][12][V] of T
  const void *gauge;     // [4][LR/2][V] of V2<T>
  double *partial;       // [nsrc][ceil(V/64)] partial Re<in, out> per wavefront, or nullptr
  const SeedState *seed; // per-source done flags, or nullptr (always compute)
  double kappa, sigma;   // out = sigma in - A in (mode 1) or A in (mode 0)
  int32_t dims[4];
  int32_t V, nsrc, nblk_site, block_begin, nblocks, mode;
  int32_t ct;            // t-slices per block of the tile kernel (0: one site per thread)
  int32_t ty, tz;        // tile kernel: tile of Lx x ty x tz sites (one thread per site)
  int32_t order;         // block order: 0 source groups outermost, 1 sites outermost
};
struct DslashBatch { DslashJob job[kMaxJobs]; int32_t njobs; int32_t total_blocks; };

struct ScalarJob {
  SeedState *seed; ShiftState *shift;
  const double *partial; // partial sums to reduce (pq or rr)
  int32_t nblk;          // partials per source
  int32_t nsrc, nshift, maxiter, block_begin;
  double tol;
  // in-loop moments (shift scalars only): g[l][k][j] = mcoef[k][j] alpha_j for the
  // shifts updated this iteration, 0 otherwise; rows k < nmom of [nsrc][32][nshift]
  const double2 *mcoef;
  double2 *mg;
  int32_t nmom, pad;
};
constexpr int kMomRows = 32;  // rows of g per source (the largest moment count)
// Element-wise pass over nsrc vectors of n complex entries of one problem.
struct VecJob {
  void *a; void *b; void *c; void *d; void *e;   // meaning depends on the kernel
  double *partial;       // [nsrc][nblk_vec]
  SeedState *seed;       // [nsrc]
  ShiftState *shift;     // [nsrc][nshift]
  int64_t n;             // complex entries per vector (12 V)
  int32_t nsrc, nshift, nblk_vec, block_begin, nblocks, wbatch;
  int32_t border;        // fused shift update: 0 shift batches outermost, 1 entry chunks outermost
  int32_t nmom;          // moments accumulated inside the solve (0: none)
  int32_t nblk_mom;      // blocks per source of the in-loop moment kernel
  // seed residual update only: > 0 = the step length is formed in the kernel from
  // this many <p, Bp> partials per source at pq_partial (no separate alpha kernel)
  int32_t npq;
  const double *pq_partial;
};
struct VecBatch { VecJob job[kMaxJobs]; int32_t njobs; int32_t total_blocks; };

// Scalar kernels: one block per (job, source).
struct ScalarBatch { ScalarJob job[kMaxJobs]; int32_t njobs; int32_t total_blocks; };

__device__ __forceinline__ int find_job(const int32_t *begins, int njobs, int b) {
  int j = 0;
  for (int k = 1; k < njobs; ++k) if (b >= begins[k]) j = k;
  return j;
}

// ---- launchers (defined in the .hip files) ---------------------------------
// dslash.hip
// nr: sources per thread (1, 2, 4); bs: sites per block (64, 128, 256).
// ct = -1: the direction-split kernel (64 sites per block, nr <= 2), nblk_site =
// ceil(V / 64); ct = 0: one thread per site, each job's nblk_site = ceil(V / bs); ct > 0: the
// tile kernel with every job's (ct, ty, tz) equal (ty | Ly, tz | Lz, Lx ty tz a
// multiple of 64 up to 1024, bs unused), nblk_site = (Ly / ty)(Lz / tz) ceil(Lt / ct).
// Blocks per job: nblk_site * ceil(nsrc / nr).
void launch_dslash(const DslashBatch &b, int prec /*0 fp64, 1 fp32*/, int nr, int lr, int bs,
                   int xcd_remap, int ct, hipStream_t st);
// vec.hip
void launch_seed_alpha(const ScalarBatch &b, hipStream_t st);
void launch_shift_scalars(const ScalarBatch &b, hipStream_t st);
void launch_seed_r_update(const VecBatch &b, int prec, hipStream_t st);
// prec: shift vectors (0 FP64, 1 FP32); seed_prec: seed r and p (0 FP64, 1 FP32);
// unroll: shifts whose loads are issued together (1, 2, 4); nt: non-temporal access
void launch_shift_update(const VecBatch &b, int prec, int seed_prec, int fold, int unroll, int nt,
                         hipStream_t st);
void launch_reliable_residual(const VecBatch &b, hipStream_t st);
// Shift update with the moment sums accumulated in the loop (no stored x_j).
// job: a = moments S (column k L + l of n entries), b = shift slots (p_j),
// c = seed r, d = seed p (FP64), e = g[l][k][j] = c[k][j] alpha_j of this
// iteration ([nsrc][kMomRows][nshift], written by the shift-scalar kernel; rows
// from nmom on stay zero).
constexpr int kMomBlock = 256;   // entries (threads) per block of the in-loop moment kernel
void launch_shift_moments(const VecBatch &b, int prec, int nmom_max, hipStream_t st);
void launch_fold_seed(const VecBatch &b, hipStream_t st);
void launch_fold_shifts(void *y, void *W, int64_t n, int nslots, hipStream_t st);
void launch_init_shifts(void *y, void *W, const void *v, int64_t n, int nsrc, int nshift, hipStream_t st);
void launch_moments_strided(const void *y, int nsrc, int nshift, const double *c_dev, int nmom, void *s,
                            int64_t n, int64_t sl, int64_t sk, hipStream_t st);
// y: [nsrc] blocks of y_stride_l vectors, the first nshift of each used
void launch_moments_strided2(const void *y, int nsrc, int nshift, int64_t y_stride_l, const double *c_dev, int nmom,
                             void *s, int64_t n, int64_t sl, int64_t sk, hipStream_t st);
void launch_to_fp32(const void *src64, void *dst32, void *zero32, int64_t n, hipStream_t st);
void launch_cast(const void *src, int src_prec, void *dst, int dst_prec, int64_t n, hipStream_t st);
void launch_pack(const void *canon, void *planar, int prec, int nsrc, int V, hipStream_t st);
void launch_unpack(const void *planar, int prec, void *canon, int nsrc, int V, hipStream_t st);
void launch_norm2_partial(const void *x, int64_t n, int nvec, double *partial, int nblk, hipStream_t st);
void launch_true_residual(const void *v, const void *y, const void *Ay, const double *z,
                          int64_t n, int nvec, double *partial, int nblk, hipStream_t st);
void launch_moments(const void *y, int nsrc, int nshift, const double *c_dev, int nmom,
                    void *s, int64_t n, hipStream_t st);
void launch_vdot_block(const void *V, int nv, const void *Y, int ny, int64_t n, double *partial,
                       int nblk, hipStream_t st);
// dense.hip: tall-skinny products (FP64 complex)
void launch_gemm_cn(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nb,
                    int64_t n, double *partial, int nchunk, hipStream_t st);
void launch_gemm_nn(const void *A, int64_t lda, int na, const double *T_dev, int nb,
                    void *C, int64_t ldc, int64_t n, hipStream_t st);
void launch_colscale(void *A, int64_t lda, int na, const double *scale_dev, int64_t n, hipStream_t st);
void launch_resid_cols(const void *AX, const void *X, int64_t ld, int ncol, const double *lam_dev,
                       int64_t n, double *partial, int nchunk, hipStream_t st);
void launch_reduce_partials(const double *partial, int nchunk, int nout, double *out, hipStream_t st);

// dense_host.cpp: Hermitian eigen-decomposition (cyclic Jacobi), column-major
// complex matrices as interleaved doubles. Eigenvalues ascending.
void herm_eig(int n, const double *A, double *evals, double *evecs);

}  // namespace sscg
