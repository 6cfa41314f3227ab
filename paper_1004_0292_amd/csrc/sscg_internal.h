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

struct sscg_ctx;

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

// ---- raw buffer access ------------------------------------------------------
// Loads and stores through a buffer resource: base address and size in bytes in
// scalar registers, a 32-bit per-lane byte offset and a scalar byte offset. A lane
// whose offset lies at or past the size reads zero and writes nothing, with no memory
// access. AUX = 2 marks the access non-temporal.

// A value the same on every lane (a scalar offset, a resource word); readfirstlane
// states it, so the compiler keeps it in scalar registers also where it meets per-lane
// branches (a resource the compiler takes for per-lane is used lane group by lane group).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int nbytes) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  void *q = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, uni(nbytes), 0x00020000);
}

template <typename T, int AUX = 0> struct BufIO;
template <int AUX> struct BufIO<double, AUX> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ double2 ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, uni(soff), AUX));
    return make_double2(v.x, v.y);
  }
  static __device__ __forceinline__ void st(double2 x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    v2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, voff, uni(soff), AUX);
  }
};
template <int AUX> struct BufIO<float, AUX> {
  typedef float v2 __attribute__((ext_vector_type(2)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float2 ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, uni(soff), AUX));
    return make_float2(v.x, v.y);
  }
  static __device__ __forceinline__ void st(float2 x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    v2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, uni(soff), AUX);
  }
};

// ---- solver state (device memory) ------------------------------------------
// The shift update kernel forms the scalars of its iteration itself (every block
// from the same inputs, so every block gets the same values) and may not change
// what its other blocks read; it stages the new values ("_n" fields), and an extra
// block of the next iteration's dslash launch commits them (commit_states below), or
// a commit launch does before the host reads the state.
// Per source: the seed CG scalars of (sigma I - A) x = v.
struct SeedState {
  double rho;        // <r_k, r_k>
  double alpha;      // alpha_k of the current iteration
  double alpha_prev; // alpha_{k-1} (1 before the first iteration)
  double beta_prev;  // beta_{k-1} (0 before the first iteration)
  double vnorm;      // ||v||
  double maxres;     // max over active shifts of ||r_j|| / ||v|| after the last update
  double rho_n;      // staged: rho_{k+1}
  double beta_n;     // staged: beta_k
  int32_t iters;     // completed iterations
  int32_t done;      // 1: no more work for this source
  int32_t status;    // SSCG_OK / SSCG_ENOTCONV / SSCG_EBREAKDOWN
  int32_t nactive;   // shifts still iterating
  int32_t pending;   // 1: alpha_k of the current iteration is set (no breakdown)
  int32_t staged;    // 1: the _n fields hold an update not yet committed
  int32_t brk_n;     // staged: rho_{k+1} or beta_k not finite
  int32_t maxiter;   // iteration limit
};
// Per (source, shift): the scalars of shift j (s_j = z_j - sigma).
struct ShiftState {
  double2 s;
  double2 pi_prev, pi_cur;   // pi_{j,k-1}, pi_{j,k}
  double2 pi_n;              // staged: pi_{j,k+1}
  double res_n;              // staged: sqrt(rho_{k+1}) / |pi_{j,k+1}| / tscale
  double tscale;             // this shift's tolerance multiplier (1: the common tol)
  int32_t active;            // still iterating (before this iteration's decision)
  int32_t frz_n;             // staged: freezes after this iteration's update
  int32_t conv_iter;         // iteration after which it froze, -1 if not yet
  int32_t pad;
};

// Scalars of one (source, shift) pair for the iteration, formed once per iteration by
// the table kernel of the in-loop moment update: alpha_{j,k}, beta_{j,k}, 1/pi_{j,k+1}
// and whether the shift is updated. The moment coefficients g_{kj} = c_{kj} alpha_{j,k}
// follow the table in the same buffer, kMomRows per shift (zero beyond the moments
// summed). Every block of the update reads them at wavefront-uniform addresses.
struct ShiftTab {
  double2 a, b, ipi;
  int32_t upd, pad;
};

// Scalars of one shift in iteration k (Sec. 2.2): from alpha_k, beta_k,
// c = alpha_k beta_{k-1} / alpha_{k-1}, sqrt(rho_{k+1}) and the committed pi values,
//   pi_{j,k+1} = (1 + c + alpha_k s_j) pi_{j,k} - c pi_{j,k-1},
//   alpha_{j,k} = alpha_k pi_{j,k}/pi_{j,k+1},  beta_{j,k} = (pi_{j,k}/pi_{j,k+1})^2 beta_k,
// and the freeze test sqrt(rho_{k+1}) / |pi_{j,k+1}| / tscale <= thr. A frozen shift
// (inactive) gets upd = 0 and zero coefficients.
struct ShiftStep {
  double2 a, b, ipi, pn;
  double res;
  int upd, frz;
};
__device__ __forceinline__ double2 cdiv_smith(double2 a, double2 b) {  // Smith's division a / b
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    const double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ ShiftStep shift_step(const ShiftState &H, double alpha, double beta, double c, double sq,
                                                double thr) {
  ShiftStep o;
  o.a = o.b = o.ipi = o.pn = make_double2(0.0, 0.0);
  o.res = 0.0;
  o.upd = o.frz = 0;
  if (!H.active) return o;
  const double2 pc = H.pi_cur, pp = H.pi_prev, s = H.s;
  const double2 f = make_double2(1.0 + c + alpha * s.x, alpha * s.y);
  double2 pn = cmul(f, pc);
  pn.x -= c * pp.x;
  pn.y -= c * pp.y;
  const double2 ratio = cdiv_smith(pc, pn);
  o.a = make_double2(alpha * ratio.x, alpha * ratio.y);
  const double2 r2 = cmul(ratio, ratio);
  o.b = make_double2(beta * r2.x, beta * r2.y);
  o.ipi = cdiv_smith(make_double2(1.0, 0.0), pn);
  o.pn = pn;
  o.res = sq / hypot(pn.x, pn.y) / H.tscale;
  o.upd = 1;
  o.frz = o.res <= thr;
  return o;
}

// Commit of the staged iteration of every source of a problem, run by one block
// (one wavefront per source; full wavefronts only): pi_{j,k-1} <- pi_{j,k} <-
// pi_{j,k+1} for the shifts that were active, freezing, the seed scalars, the count
// of active shifts and the largest active residual, and the end of the source's run
// (all shifts frozen, breakdown, or the iteration limit).
__device__ inline void commit_states(SeedState *seed, ShiftState *shift, int nsrc, int nshift) {
  const int nw = blockDim.x / 64, w = threadIdx.x / 64, lane = threadIdx.x & 63;
  if (w >= nw) return;
  for (int l = w; l < nsrc; l += nw) {
    SeedState &S = seed[l];
    if (!S.staged) continue;  // uniform over the wavefront
    int nact = 0;
    double mr = 0.0;
    for (int j = lane; j < nshift; j += 64) {
      ShiftState &H = shift[(size_t)l * nshift + j];
      if (!H.active) continue;
      H.pi_prev = H.pi_cur;
      H.pi_cur = H.pi_n;
      if (H.frz_n) {
        H.active = 0;
      } else {
        nact += 1;
        mr = fmax(mr, H.res_n / S.vnorm);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      nact += __shfl_xor(nact, off, 64);
      mr = fmax(mr, __shfl_xor(mr, off, 64));
    }
    if (lane == 0) {
      S.alpha_prev = S.alpha;
      S.beta_prev = S.beta_n;
      S.rho = S.rho_n;
      S.iters += 1;
      S.nactive = nact;
      S.maxres = mr;
      S.pending = 0;
      if (S.brk_n) {
        S.status = -5;  // SSCG_EBREAKDOWN
        S.done = 1;
      } else if (nact == 0) {
        S.status = 0;
        S.done = 1;
      } else if (S.iters >= S.maxiter) {
        S.status = -4;  // SSCG_ENOTCONV
        S.done = 1;
      }
      S.staged = 0;
    }
  }
}

// ---- job tables -------------------------------------------------------------
// A grouped launch covers up to kMaxJobs problems; block b belongs to the job
// whose [block_begin, block_begin + nblocks) range contains it.
struct DslashJob {
  const void *in;        // planar [nsrc][12][V] of T
  void *out;             // planar [nsrc][12][V] of T
  const void *gauge;     // [4][LR/2][V] of V2<T>
  double *partial;       // [nsrc][ceil(V/64)] partial Re<in, out> per wavefront, or nullptr
  SeedState *seed;       // per-source done flags, or nullptr (always compute)
  ShiftState *shift;     // solve loop: the states the launch's commit block commits (or nullptr)
  int32_t nshift, pad0;
  double kappa, sigma;   // out = sigma in - A in (mode 1) or A in (mode 0)
  int32_t dims[4];
  int32_t V, nsrc, nblk_site, block_begin, nblocks, mode;
  int32_t ct;            // t-slices per block of the tile kernel (0: one site per thread)
  int32_t ty, tz;        // tile kernel: tile of Lx x ty x tz sites (one thread per site)
  int32_t order;         // block order: 0 source groups outermost, 1 sites outermost
};
// commit = 1: one block more than total_blocks, which commits the staged states of
// the jobs with a shift table (solve loop)
struct DslashBatch { DslashJob job[kMaxJobs]; int32_t njobs; int32_t total_blocks; int32_t commit; int32_t pad; };

// Step length kernel (large lattices): one block per (job, source).
struct ScalarJob {
  SeedState *seed;
  const double *partial; // <p, Bp> partials to reduce
  int32_t nblk;          // partials per source
  int32_t nsrc, block_begin, pad;
};
constexpr int kMomRows = 32;  // largest moment count accumulated inside the solve
constexpr int kMaxWBatch = 64;  // largest shift batch of the fused shift update
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
  // shift update (and its in-loop moment form): the scalars of the iteration are
  // formed from the nrr <r, r> partials per source at rr_partial; tol is the
  // common tolerance; mcoef[k][j] the moment coefficients c_kj; identity = 1 runs
  // the update with alpha_j = 0, beta_j = 1, 1/pi_j = 0 and writes no state
  // (launch-shape timing)
  const double *rr_partial;
  const double2 *mcoef;
  double tol;
  int32_t nrr, identity;
  // block form of the in-loop moment update: block length (0: the per-iteration form).
  // The seed residuals of a block live in a ring of `ring` slots of nsrc vectors each
  // (slot s of source l at complex offset (s nsrc + l) n of the ring buffer); within a
  // block, iteration s writes r_{s+1} to slot s, and r_0 of a block is the previous
  // block's last residual, in slot ring - 1.
  int32_t ring, pad_ring;
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
// commit of the staged states of every job with a shift table (one block per job)
void launch_commit(const DslashBatch &b, hipStream_t st);
void launch_seed_r_update(const VecBatch &b, int prec, hipStream_t st, int slot = 0);
// prec: shift vectors (0 FP64, 1 FP32); seed_prec: seed r and p (0 FP64, 1 FP32);
// unroll: shifts whose loads are issued together (1, 2, 4); nt: non-temporal access
void launch_shift_update(const VecBatch &b, int prec, int seed_prec, int fold, int unroll, int nt,
                         hipStream_t st);
void launch_reliable_residual(const VecBatch &b, hipStream_t st);
// Shift update with the moment sums accumulated in the loop (no stored x_j).
// job: a = moments S (column k L + l of n entries), b = shift slots (p_j),
// c = seed r, d = seed p (FP64); mcoef [nmom][nshift].
constexpr int kMomBlock = 256;   // entries (threads) per block of the in-loop moment kernel
// In-loop moments in two launches: the table kernel (one thread per (source, shift),
// job e = table buffer of nsrc * nshift ShiftTab records followed by nsrc * nshift *
// kMomRows coefficients) stages the iteration's scalars; the update kernel (one entry
// per thread) reads them with uniform loads. Blocks per source of the table kernel:
// ceil(nshift / kBlock); of the update: nblk_mom.
void launch_shift_table(const VecBatch &b, hipStream_t st, int slot = 0);
// ub: shifts whose loads are issued together (1, 2, 4)
void launch_shift_moments_tab(const VecBatch &b, int prec, int nmom_max, int ub, int pf, hipStream_t st);
inline size_t shift_table_bytes(int nsrc, int nshift) {
  return (size_t)nsrc * nshift * (sizeof(ShiftTab) + (size_t)kMomRows * sizeof(double2));
}
// Block form (VecJob::ring = B > 0, B in {4, 8, 16, 24, 32}): the table kernel writes the
// iteration's record of every (source, shift) into slot s of a history of B records
// (not-updated records: alpha 0, beta 1, 1/pi 0); after the B-th iteration (and once
// after the loop) the compose kernel folds the history into one linear map per shift
// (BlkShift plus B coefficients D) and the moment coefficients G (rows of the g area)
// and H, and resets the history; the pass kernel applies them in one sweep over the
// entries. Regions of the table buffer, byte offsets:
//   hist  ShiftTab [nsrc][nshift][B]      records of the block
//   g     double2 [nsrc][nshift][kMomRows] G_kj (zero beyond the moments summed)
//   comp  BlkShift [nsrc][nshift]          C_j and the flags
//   d     double2 [nsrc][nshift][B]        D_j(B, m), m = 1..B
//   h     double2 [nsrc][kMomRows][B]      H_km, m = 1..B (the last is zero)
//   e     double2 [nsrc][nshift][B]        per-shift terms of H (work area)
//   any   int32 [nsrc]                     bit 0: a shift of the source moved in the block,
//                                          bit 1: a shift is still active at its end,
//                                          bit 2: the block is the source's first (every
//                                          p_j(0) is v, read from v itself)
//   fresh int32 [nsrc]                     1 until the first block's composition
//   cnt   uint64 [2][5]                    sweep counts per direction precision (0 FP64,
//                                          1 FP32), summed over the solve: moment-kernel
//                                          (source, block) runs and directions read,
//                                          direction-kernel runs, directions read and
//                                          directions written
struct BlkShift {
  double2 c;       // C_j(B)
  int32_t any;     // updated in at least one iteration of the block (p_j(0) is read)
  int32_t st;      // still active at the end of the block (p_j(B) is written)
  int32_t pad[2];
};
struct BlkLayout {
  size_t hist, g, comp, d, h, e, any, fresh, cnt, total;
};
constexpr int kBlkCnt = 5;  // counts per precision in the cnt region
__host__ __device__ inline BlkLayout blk_layout(int nsrc, int nshift, int B) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t sn = (size_t)nsrc * nshift;
  BlkLayout o;
  o.hist = 0;
  o.g = up(o.hist + sn * B * sizeof(ShiftTab));
  o.comp = up(o.g + sn * kMomRows * sizeof(double2));
  o.d = up(o.comp + sn * sizeof(BlkShift));
  o.h = up(o.d + sn * B * sizeof(double2));
  o.e = up(o.h + (size_t)nsrc * kMomRows * B * sizeof(double2));
  o.any = up(o.e + sn * B * sizeof(double2));
  o.fresh = up(o.any + (size_t)nsrc * sizeof(int32_t));
  o.cnt = up(o.fresh + (size_t)nsrc * sizeof(int32_t));
  o.total = up(o.cnt + 2 * kBlkCnt * sizeof(unsigned long long));
  return o;
}
// history records set to the identity, every source marked fresh, the sweep counts
// zero (start of a solve; the shift directions are not written: a source's first
// sweep reads v instead)
void launch_blk_init(void *tab, int nsrc, int nshift, int B, hipStream_t st);
// p <- r_{s+1} + beta_k p (the seed direction, every iteration of the block form);
// job a = residual ring, d = seed p; one source per nblk_vec blocks like the seed passes
void launch_seed_p_update(const VecBatch &b, int slot, hipStream_t st);
// compose: one block per source (total_blocks = sources of all jobs); job e = table;
// prec: precision of the shift directions (selects the counts it adds to)
void launch_blk_compose(const VecBatch &b, int B, int prec, hipStream_t st);
// pass: the in-loop moment kernel's grid; job a = moments, b = shift directions
// (chunk-blocked), c = residual ring, d = the sources v (planar FP64), e = table
void launch_blk_pass(const VecBatch &b, int prec, int nmom_max, int B, hipStream_t st);
void launch_fold_seed(const VecBatch &b, hipStream_t st);
void launch_fold_shifts(void *y, void *W, int64_t n, int nslots, hipStream_t st);
void launch_init_shifts(void *y, void *W, const void *v, int64_t n, int nsrc, int nshift, hipStream_t st);
// in-loop moment form: p_j = v in the chunk-blocked layout of the shift directions
// (entry 64 c + q of shift j of source l at double2 ((l ceil(n/64) + c) N + j) 64 + q),
// and the in-place FP32 switch of that layout (each 64-entry run's float2 in its
// first half)
void launch_init_shifts_blocked(void *W, const void *v, int64_t n, int nsrc, int nshift, hipStream_t st);
void launch_blocked_to_fp32(void *W, int64_t n, int nsrc, int nshift, hipStream_t st);
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
// dense.hip: tall-skinny products (FP64 complex). gemm_cn with herm = 1 (Hermitian
// product, na = nb) computes the 64 x 64 output tiles on and above the diagonal only
// (the entries below are not written); gemm_nn with upper = 1 takes T upper triangular.
void launch_gemm_cn(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nb,
                    int64_t n, double *partial, int nchunk, int herm, hipStream_t st);
void launch_gemm_nn(const void *A, int64_t lda, int na, const double *T_dev, int nb,
                    void *C, int64_t ldc, int64_t n, int upper, hipStream_t st);
// output tiles (blocks per chunk) of launch_gemm_cn
int gemm_cn_tiles(int na, int nb, int herm);
void launch_colscale(void *A, int64_t lda, int na, const double *scale_dev, int64_t n, hipStream_t st);
void launch_resid_cols(const void *AX, const void *X, int64_t ld, int ncol, const double *lam_dev,
                       int64_t n, double *partial, int nchunk, hipStream_t st);
void launch_reduce_partials(const double *partial, int nchunk, int nout, double *out, hipStream_t st);

// api.cpp: y = A x for nsrc canonical spinors through caller-given planar staging
// buffers (each nsrc * 12 V complex numbers of the precision), on the context's
// stream; tune = false uses an already tuned or the default launch shape and never
// times one (no events, no allocation). The checks and accessors serve entry points
// defined in other files.
int apply_A_staged(sscg_ctx *c, const void *x, void *y, int nsrc, int prec, void *stage_in, void *stage_out,
                   bool tune);
int context_check_apply(sscg_ctx *c, const void *x, const void *y, int nsrc, int prec, size_t *bytes_each);
int context_device(const sscg_ctx *c);
int context_fail(sscg_ctx *c, int code, const char *msg);

// dense_host.cpp: Hermitian eigen-decomposition (Householder tridiagonalisation and
// implicit symmetric QR with Wilkinson shifts), column-major complex matrices as
// interleaved doubles. Eigenvalues ascending. Returns false if the QR iteration did
// not converge within its step limit (outputs then undefined). Declared in
// host_math.h.

}  // namespace sscg
