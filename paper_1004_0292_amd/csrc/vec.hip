// Streaming and scalar kernels of the shifted CG method (Sec. 2.2) and the moment
// sums (eq. 2).
//
// Per iteration k of the seed system B x = v, B = sigma I - A, for every source:
//   dslash        q = B p, partial Re<p, q>; its first block commits the state
//                 staged by the previous iteration                (dslash.hip)
//   seed_alpha    alpha_k = rho_k / <p, q> (large lattices; on small ones the
//                 residual update forms it itself)
//   seed_r_update r <- r - alpha_k q, partial <r, r>
//   shift_update  every block forms rho_{k+1}, beta_k and, for the shifts of its
//                 batch (s_j = z_j - sigma),
//                 pi_{j,k+1} = (1 + c + alpha_k s_j) pi_{j,k} - c pi_{j,k-1},
//                 c = alpha_k beta_{k-1} / alpha_{k-1},
//                 alpha_{j,k} = alpha_k pi_{j,k}/pi_{j,k+1},
//                 beta_{j,k} = (pi_{j,k}/pi_{j,k+1})^2 beta_k,
//                 and the freeze test sqrt(rho_{k+1}) / |pi_{j,k+1}| <= tol ||v||;
//                 then x_j += alpha_{j,k} p_j, p_j <- r/pi_{j,k+1} + beta_{j,k} p_j
//                 for every shift active in this iteration, and p <- r + beta_k p;
//                 the seed residual r is read once per batch of shifts. The new
//                 scalars are staged for the commit.
// Every reduction writes one partial per block and the consumer sums them in a
// fixed order, so results do not depend on scheduling.
#include <cstddef>

#include "sscg_internal.h"

namespace sscg {

static constexpr int kEpt = 2;  // complex entries per thread in streaming kernels
static_assert(kBlock >= kMaxWBatch, "the shift update forms one shift's scalars per thread");

template <int NW>
__device__ __forceinline__ double block_sum_all(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += sh[i];
  __syncthreads();
  return t;  // valid in every thread
}
template <int NW>
__device__ __forceinline__ double block_max_all(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t = fmax(t, sh[i]);
  __syncthreads();
  return t;
}

template <typename J>
__device__ __forceinline__ int job_of(const J *jobs, int njobs, int b) {
  int j = 0;
  for (int k = 1; k < njobs; ++k) if (b >= jobs[k].block_begin) j = k;
  return j;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void seed_alpha_kernel(ScalarBatch B) {
  __shared__ double red[kBlock / 64];
  const int b = blockIdx.x;
  const ScalarJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int l = b - J.block_begin;
  SeedState &S = J.seed[l];
  const int done = S.done;
  __syncthreads();
  if (threadIdx.x == 0) S.pending = 0;
  if (done) return;
  double v = 0.0;
  const double *p = J.partial + (size_t)l * J.nblk;
  for (int i = threadIdx.x; i < J.nblk; i += kBlock) v += p[i];
  const double pq = block_sum_all<kBlock / 64>(v, red);
  if (threadIdx.x == 0) {
    if (pq == 0.0 || !isfinite(pq)) {
      S.status = -5;  // SSCG_EBREAKDOWN
      S.done = 1;
    } else {
      S.alpha = S.rho / pq;
      S.pending = 1;
    }
  }
}

// Commit of the staged states outside the solve loop's dslash (before the host
// reads them): block b commits job b.
__global__ __launch_bounds__(kBlock) void commit_kernel(DslashBatch B) {
  const DslashJob &J = B.job[blockIdx.x];
  if (J.shift && J.seed) commit_states(J.seed, J.shift, J.nsrc, J.nshift);
}

// ---------------------------------------------------------------------------
// Non-temporal (streaming) loads and stores of one complex number.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ double2 ldc(const double2 *p) {
  if constexpr (NT) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2 *>(p));
    return make_double2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ float2 ldc(const float2 *p) {
  if constexpr (NT) {
    const nf2 v = __builtin_nontemporal_load(reinterpret_cast<const nf2 *>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ void stc(double2 *p, double2 v) {
  if constexpr (NT) {
    nd2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nd2 *>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void stc(float2 *p, float2 v) {
  if constexpr (NT) {
    nf2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nf2 *>(p));
  } else {
    *p = v;
  }
}

// r <- r - alpha q (and x_part += alpha p in the FP32 phase); partial <r, r>.
// job: a = r, b = q, c = x_part (or null), d = p. With a residual ring (block form of
// the in-loop update) the new r goes to ring slot `slot` and the old one is read from
// the slot before it (cyclically), instead of updating r in place.
template <typename T>
__global__ __launch_bounds__(kBlock) void seed_r_update_kernel(VecBatch B, int slot) {
  using C = V2<T>;
  __shared__ double red[kBlock / 64];
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int l = lb / J.nblk_vec, vb = lb - l * J.nblk_vec;
  SeedState &S = J.seed[l];
  if (S.done) return;
  C *r = reinterpret_cast<C *>(J.a) + (size_t)l * J.n;
  const C *rin = r;
  if (J.ring > 0) {
    const int sin = slot == 0 ? J.ring - 1 : slot - 1;
    rin = reinterpret_cast<const C *>(J.a) + ((size_t)sin * J.nsrc + l) * J.n;
    r = reinterpret_cast<C *>(J.a) + ((size_t)slot * J.nsrc + l) * J.n;
  }
  const C *q = reinterpret_cast<const C *>(J.b) + (size_t)l * J.n;
  C *xp = J.c ? reinterpret_cast<C *>(J.c) + (size_t)l * J.n : nullptr;
  const C *p = J.d ? reinterpret_cast<const C *>(J.d) + (size_t)l * J.n : nullptr;
  // chunks of kBlock kEpt entries, strided by the source's block count (at most
  // kMaxRR blocks per source, so the consumers of the partials sum few of them); the
  // first chunk is loaded before the step length is formed, so the two latencies overlap
  const int64_t base0 = (int64_t)vb * kBlock * kEpt + threadIdx.x;
  C r0[kEpt], q0[kEpt], x0[kEpt], p0[kEpt];
#pragma unroll
  for (int e = 0; e < kEpt; ++e) {
    const int64_t i = base0 + (int64_t)e * kBlock;
    if (i < J.n) {  // streaming accesses (no vector is re-read before it leaves the caches)
      r0[e] = ldc<true>(rin + i);
      q0[e] = ldc<true>(q + i);
      if (xp) {
        x0[e] = ldc<true>(xp + i);
        p0[e] = ldc<true>(p + i);
      }
    }
  }
  double alpha64;
  if (J.npq > 0) {
    // the step length of the alpha kernel, formed by every block from the same
    // partials in the same order (so every block gets the same value); the first
    // block of the source also writes the seed state
    double v = 0.0;
    const double *pp = J.pq_partial + (size_t)l * J.npq;
    for (int t = threadIdx.x; t < J.npq; t += kBlock) v += pp[t];
    const double pq = block_sum_all<kBlock / 64>(v, red);
    const bool broke = pq == 0.0 || !isfinite(pq);
    alpha64 = broke ? 0.0 : S.rho / pq;
    if (vb == 0 && threadIdx.x == 0) {
      if (broke) {
        S.status = -5;  // SSCG_EBREAKDOWN
        S.done = 1;
      } else {
        S.alpha = alpha64;
        S.pending = 1;
      }
    }
    if (broke) return;
  } else {
    alpha64 = S.alpha;
  }
  const T alpha = (T)alpha64;
  double acc = 0.0;
  auto update = [&](int64_t i, C rv, C qv, C xv, C pv) {
    rv.x -= alpha * qv.x;
    rv.y -= alpha * qv.y;
    stc<true>(r + i, rv);
    acc += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
    if (xp) {
      xv.x += alpha * pv.x;
      xv.y += alpha * pv.y;
      stc<true>(xp + i, xv);
    }
  };
#pragma unroll
  for (int e = 0; e < kEpt; ++e) {
    const int64_t i = base0 + (int64_t)e * kBlock;
    if (i < J.n) update(i, r0[e], q0[e], x0[e], p0[e]);
  }
  const int64_t stride = (int64_t)J.nblk_vec * kBlock * kEpt;
  for (int64_t base = base0 + stride; base - threadIdx.x < J.n; base += stride) {
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < J.n)
        update(i, ldc<true>(rin + i), ldc<true>(q + i), xp ? ldc<true>(xp + i) : C{}, xp ? ldc<true>(p + i) : C{});
    }
  }
  const double tot = block_sum_all<kBlock / 64>(acc, red);
  if (threadIdx.x == 0) J.partial[(size_t)l * J.nblk_vec + vb] = tot;
}


// Fused multi-shift update. job: a = x (FP64 solution storage [nsrc][nshift][n]),
// b = shift workspace [nsrc][nshift] slots of n double2: FP64 phase p_j;
// FP32 phase p_j (first n float2) and the FP32 partial x_j (next n float2);
// c = seed r, d = seed p (both T). FOLD (FP32 phase only) also adds the partial
// and this iteration's step into the FP64 solution and clears the partial.
// U shifts are handled together: all their loads are issued before the first
// store, so a thread keeps 2 U kEpt loads in flight. NT selects streaming
// (non-temporal) access for the shift vectors, which are touched once per
// iteration.
// The block first forms the scalars of the iteration for the shifts of its batch
// (shift_step, in LDS); the first entry chunk's block of each batch stages them
// for the commit, and the first block of the source stages rho_{k+1} and beta_k.
template <typename T, typename TR, bool FOLD, int U, bool NT>
__global__ __launch_bounds__(kBlock) void shift_update_kernel(VecBatch B) {
  using C = V2<TR>;  // seed vectors r and p (TR); shift vectors in T
  __shared__ double red[kBlock / 64];
  __shared__ double2 s_a[kMaxWBatch], s_b[kMaxWBatch], s_ip[kMaxWBatch];
  __shared__ int s_up[kMaxWBatch];
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int nbatch = (J.nshift + J.wbatch - 1) / J.wbatch;
  const int per_src = nbatch * J.nblk_vec;
  const int l = lb / per_src;
  const int rem = lb - l * per_src;
  // block order: shift batches outermost (border 0) or entry chunks outermost
  // (border 1: the batches of one chunk are neighbouring blocks, so the chunk of the
  // seed residual they all read stays in L2)
  int bt, vb;
  if (J.border) {
    vb = rem / nbatch;
    bt = rem - vb * nbatch;
  } else {
    bt = rem / J.nblk_vec;
    vb = rem - bt * J.nblk_vec;
  }
  SeedState &S = J.seed[l];
  if (S.done || !S.pending) return;  // uniform over the block
  const int64_t n = J.n;
  const C *r = reinterpret_cast<const C *>(J.c) + (size_t)l * n;
  const int64_t base = (int64_t)vb * kBlock * kEpt + threadIdx.x;
  C rv[kEpt];
#pragma unroll
  for (int e = 0; e < kEpt; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
    rv[e] = i < n ? r[i] : cmk<C>(0, 0);
  }
  const int j0 = bt * J.wbatch, j1 = min(j0 + J.wbatch, J.nshift);
  double beta64 = 0.0;
  bool bad = false;
  if (J.identity) {
    for (int jj = threadIdx.x; jj < j1 - j0; jj += kBlock) {
      s_a[jj] = s_ip[jj] = make_double2(0.0, 0.0);
      s_b[jj] = make_double2(1.0, 0.0);
      s_up[jj] = 1;
    }
  } else {
    // the shift states and seed scalars are loaded before the reduction, so their
    // latency overlaps that of the partials
    const int jj0 = threadIdx.x;  // kBlock >= kMaxWBatch: one shift per thread at most
    ShiftState Hl;
    if (jj0 < j1 - j0) Hl = J.shift[(size_t)l * J.nshift + j0 + jj0];
    const double alpha = S.alpha, rho = S.rho, bprev = S.beta_prev, aprev = S.alpha_prev, vnorm = S.vnorm;
    const int it = S.iters;
    double v = 0.0;
    const double *pr = J.rr_partial + (size_t)l * J.nrr;
    for (int t = threadIdx.x; t < J.nrr; t += kBlock) v += pr[t];
    const double rho_new = block_sum_all<kBlock / 64>(v, red);
    beta64 = rho_new / rho;
    const double c = alpha * bprev / aprev;
    const double sq = sqrt(rho_new);
    const double thr = J.tol * vnorm;
    bad = !isfinite(rho_new) || !isfinite(beta64);
    const bool writer = vb == 0 && !bad;
    if (jj0 < j1 - j0) {
      const int jj = jj0;
      ShiftState &H = J.shift[(size_t)l * J.nshift + j0 + jj];
      const ShiftStep o = shift_step(Hl, alpha, beta64, c, sq, thr);
      s_a[jj] = o.a;
      s_b[jj] = o.b;
      s_ip[jj] = o.ipi;
      s_up[jj] = o.upd;
      if (writer && o.upd) {
        H.pi_n = o.pn;
        H.res_n = o.res;
        H.frz_n = o.frz;
        if (o.frz) H.conv_iter = it + 1;
      }
    }
    if (vb == 0 && bt == 0 && threadIdx.x == 0) {
      S.rho_n = rho_new;
      S.beta_n = beta64;
      S.brk_n = bad ? 1 : 0;
      S.staged = 1;
    }
  }
  __syncthreads();
  if (bad) return;  // uniform: the commit ends this source's run
  for (int j = j0; j < j1; j += U) {
    bool act[U];
    double2 a[U], bb[U], ip[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      act[u] = false;
      if (j + u < j1) {
        const int jj = j - j0 + u;
        act[u] = s_up[jj] != 0;
        a[u] = s_a[jj];
        bb[u] = s_b[jj];
        ip[u] = s_ip[jj];
      }
    }
    if constexpr (sizeof(T) == 8) {
      double2 xv[U][kEpt], pv[U][kEpt];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        const size_t slot = (size_t)l * J.nshift + j + u;
        const double2 *x = reinterpret_cast<const double2 *>(J.a) + slot * n;
        const double2 *p = reinterpret_cast<const double2 *>(J.b) + slot * n;
#pragma unroll
        for (int e = 0; e < kEpt; ++e) {
          const int64_t i = base + (int64_t)e * kBlock;
          if (i < n) {
            xv[u][e] = ldc<NT>(x + i);
            pv[u][e] = ldc<NT>(p + i);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        const size_t slot = (size_t)l * J.nshift + j + u;
        double2 *x = reinterpret_cast<double2 *>(J.a) + slot * n;
        double2 *p = reinterpret_cast<double2 *>(J.b) + slot * n;
#pragma unroll
        for (int e = 0; e < kEpt; ++e) {
          const int64_t i = base + (int64_t)e * kBlock;
          if (i < n) {
            double2 xn = xv[u][e];
            cfma(xn, a[u], pv[u][e]);
            double2 pn = cmul(ip[u], rv[e]);
            cfma(pn, bb[u], pv[u][e]);
            stc<NT>(x + i, xn);
            stc<NT>(p + i, pn);
          }
        }
      }
    } else {
      float2 xv[U][kEpt], pv[U][kEpt];
      double2 xm[FOLD ? U : 1][kEpt];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        const size_t slot = (size_t)l * J.nshift + j + u;
        const float2 *p = reinterpret_cast<const float2 *>(reinterpret_cast<const double2 *>(J.b) + slot * n);
        const float2 *xp = p + n;
#pragma unroll
        for (int e = 0; e < kEpt; ++e) {
          const int64_t i = base + (int64_t)e * kBlock;
          if (i < n) {
            pv[u][e] = ldc<NT>(p + i);
            xv[u][e] = ldc<NT>(xp + i);
            if constexpr (FOLD) xm[u][e] = ldc<NT>(reinterpret_cast<const double2 *>(J.a) + slot * n + i);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        const size_t slot = (size_t)l * J.nshift + j + u;
        float2 *p = reinterpret_cast<float2 *>(reinterpret_cast<double2 *>(J.b) + slot * n);
        float2 *xp = p + n;
        const float2 af = make_float2((float)a[u].x, (float)a[u].y);
        float2 rf[kEpt];
#pragma unroll
        for (int e = 0; e < kEpt; ++e) rf[e] = make_float2((float)rv[e].x, (float)rv[e].y);
        const float2 bf = make_float2((float)bb[u].x, (float)bb[u].y);
        const float2 pf = make_float2((float)ip[u].x, (float)ip[u].y);
#pragma unroll
        for (int e = 0; e < kEpt; ++e) {
          const int64_t i = base + (int64_t)e * kBlock;
          if (i < n) {
            float2 pn = cmul(pf, rf[e]);
            cfma(pn, bf, pv[u][e]);
            stc<NT>(p + i, pn);
            if constexpr (FOLD) {
              double2 m = xm[u][e];
              m.x += (double)xv[u][e].x;
              m.y += (double)xv[u][e].y;
              cfma(m, a[u], make_double2(pv[u][e].x, pv[u][e].y));
              stc<NT>(reinterpret_cast<double2 *>(J.a) + slot * n + i, m);
              stc<NT>(xp + i, make_float2(0.f, 0.f));
            } else {
              float2 xn = xv[u][e];
              cfma(xn, af, pv[u][e]);
              stc<NT>(xp + i, xn);
            }
          }
        }
      }
    }
  }
  if (bt == 0) {
    const TR beta = (TR)beta64;
    C *p = reinterpret_cast<C *>(J.d) + (size_t)l * n;
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < n) {
        C pv = p[i];
        pv.x = rv[e].x + beta * pv.x;
        pv.y = rv[e].y + beta * pv.y;
        p[i] = pv;
      }
    }
  }
}

// Moment sums accumulated inside the solve (eq. 2 summed as the solve runs): for every
// shift updated in an iteration, the step alpha_j p_j that would be added to x_j is
// added to every moment instead, s_{k,l} += c[k][j] alpha_j p_j, and p_j advances as
// usual; the solutions x_j are never stored. Two launches per iteration. The table
// kernel forms, once per iteration and
// (source, shift), the scalars of shift_step from the seed scalars and the new
// <r, r> (summed from the residual update's partials by every block in the same
// order), writes a_j, b_j, 1/pi_j, the update flag and g_kj = c_kj a_j for k < kMomRows
// (zero beyond the moments summed) to the table, and stages the shift state for the
// commit (one writer per shift; the first block of a source stages the seed scalars).
// In the block form (J.ring = B > 0) the record goes to slot `slot` of the source's
// history of B records instead (a shift not updated gets the identity record alpha 0,
// beta 1, 1/pi 0; the flag word after upd holds the freeze), and no coefficients
// are written: the compose kernel forms them for the whole block.
__global__ __launch_bounds__(kBlock) void shift_table_kernel(VecBatch B, int slot) {
  __shared__ double red[kBlock / 64];
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int nch = (J.nshift + kBlock - 1) / kBlock;
  const int l = lb / nch, ch = lb - l * nch;
  SeedState &S = J.seed[l];
  if (S.done || !S.pending) return;  // uniform over the block
  const int N = J.nshift;
  const int j = ch * kBlock + threadIdx.x;
  ShiftState Hl;
  if (j < N) Hl = J.shift[(size_t)l * N + j];
  const double alpha = S.alpha, rho = S.rho, bprev = S.beta_prev, aprev = S.alpha_prev, vnorm = S.vnorm;
  const int it = S.iters;
  double v = 0.0;
  const double *pr = J.rr_partial + (size_t)l * J.nrr;
  for (int t = threadIdx.x; t < J.nrr; t += kBlock) v += pr[t];
  const double rho_new = block_sum_all<kBlock / 64>(v, red);
  const double beta = rho_new / rho;
  const double cc = alpha * bprev / aprev;
  const double sq = sqrt(rho_new);
  const double thr = J.tol * vnorm;
  const bool bad = !isfinite(rho_new) || !isfinite(beta);
  if (ch == 0 && threadIdx.x == 0) {
    S.rho_n = rho_new;
    S.beta_n = beta;
    S.brk_n = bad ? 1 : 0;
    S.staged = 1;
  }
  if (j >= N) return;
  ShiftTab *tab = reinterpret_cast<ShiftTab *>(J.e) + (size_t)l * N;
  double2 *g = reinterpret_cast<double2 *>(reinterpret_cast<ShiftTab *>(J.e) + (size_t)J.nsrc * N) +
               ((size_t)l * N + j) * kMomRows;
  ShiftStep o;
  if (bad) {
    o.a = o.b = o.ipi = o.pn = make_double2(0.0, 0.0);
    o.upd = o.frz = 0;
  } else {
    o = shift_step(Hl, alpha, beta, cc, sq, thr);
  }
  ShiftTab t;
  t.a = o.a;
  t.b = o.b;
  t.ipi = o.ipi;
  t.upd = o.upd;
  t.pad = 0;
  if (J.ring > 0) {
    if (!o.upd) t.b = make_double2(1.0, 0.0);
    t.pad = o.upd && o.frz;
    const BlkLayout lay = blk_layout(J.nsrc, N, J.ring);
    ShiftTab *hist = reinterpret_cast<ShiftTab *>(reinterpret_cast<char *>(J.e) + lay.hist);
    hist[((size_t)l * N + j) * J.ring + slot] = t;
  } else {
    tab[j] = t;
#pragma unroll 4
    for (int k = 0; k < kMomRows; ++k)
      g[k] = (o.upd && k < J.nmom) ? cmul(J.mcoef[(size_t)k * N + j], o.a) : make_double2(0.0, 0.0);
  }
  if (o.upd) {
    ShiftState &H = J.shift[(size_t)l * N + j];
    H.pi_n = o.pn;
    H.res_n = o.res;
    H.frz_n = o.frz;
    if (o.frz) H.conv_iter = it + 1;
  }
}

// Shift directions of the in-loop moment form, chunk-blocked: entry i = 64 c + q of
// shift j of source l is double2 number ((l nch + c) N + j) 64 + q of the slot
// buffer (nch = ceil(n / 64), entries past n are padding). A wavefront that owns one
// chunk of 64 entries then walks one contiguous run of N kilobytes over its shifts,
// instead of N runs a whole vector apart (about 10 % more of the HBM peak for the
// streaming pattern of this update). In the FP32 phase a chunk holds its 64 float2 in
// its first half (the chunk stride stays 1 KB), so the switch converts each chunk in
// place.
__device__ __forceinline__ size_t blk_chunk(int l, int64_t c, int j, int64_t nch, int N) {
  return (((size_t)l * nch + c) * N + j) * 64;  // double2 index of chunk (l, c, j)
}

// The update of the table form: one thread per entry of one source loops over the
// shifts (UB at a time), adds g_kj p_j to each of its MM moment sums (rows beyond the
// moments summed have g = 0) and advances p_j <- r / pi_j + b_j p_j for every shift
// the table marks as updated. The table and coefficients sit at addresses that are
// the same for the whole wavefront; the seed direction is advanced with the staged
// beta_k. job: a = moments, b = shift directions (chunk-blocked), c = seed r, d = seed
// p (FP64), e = the table.
// Memory: each (chunk, shift) run of 64 entries is read and written through a buffer
// resource of its own, of size zero for a shift not updated; lanes past the end get
// an offset past the size. Every load and store is therefore issued on every path (a
// masked lane or shift moves no data), so the number of memory operations in flight
// is known and the compiler waits for exactly the loads it needs. Vector loads and
// stores share one completion counter that counts down in issue order, so a load
// issued after a store is only seen complete once the store is: the moments (and the
// seed direction) are read at the start and written only at the end, and with PF = 1
// the loads of the next group of UB shifts are issued before the stores of the
// current group.
template <typename T, int MM, int UB, int PF>
__global__ __launch_bounds__(kMomBlock) void shift_moments_tab_kernel(VecBatch B) {
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int l = lb / J.nblk_mom, vb = lb - l * J.nblk_mom;
  const SeedState &S = J.seed[l];
  if (S.done || !S.pending || S.brk_n) return;  // uniform over the block
  const int64_t n = J.n;
  const int64_t nch = (n + 63) / 64;
  const int N = J.nshift;
  const int64_t i = (int64_t)vb * kMomBlock + threadIdx.x;
  const bool valid = i < n;
  const int64_t ii = valid ? i : 0;  // invalid lanes read entry 0 and store nothing
  const int64_t c = i >> 6;          // the wavefront's chunk (the same on all its lanes)
  const int q = (int)(i & 63);
  const double2 rv = reinterpret_cast<const double2 *>(J.c)[(size_t)l * n + ii];
  // the table is read-only for this kernel: read through the constant address space,
  // where the wavefront-uniform addresses become scalar loads into SGPRs (record t
  // holds a, b, ipi at doubles kRecD t .. kRecD t + 5 and the flag at int kRecI t + kUpdI)
  typedef __attribute__((address_space(4))) const double CDbl;
  typedef __attribute__((address_space(4))) const int32_t CInt;
  constexpr int kRecD = sizeof(ShiftTab) / sizeof(double), kRecI = sizeof(ShiftTab) / sizeof(int32_t);
  constexpr int kUpdI = offsetof(ShiftTab, upd) / sizeof(int32_t);
  CDbl *tabd = reinterpret_cast<CDbl *>(reinterpret_cast<uintptr_t>(J.e)) + (size_t)l * N * kRecD;
  CInt *tabi = reinterpret_cast<CInt *>(reinterpret_cast<uintptr_t>(J.e)) + (size_t)l * N * kRecI;
  CDbl *gtab = reinterpret_cast<CDbl *>(reinterpret_cast<uintptr_t>(reinterpret_cast<const ShiftTab *>(J.e) +
                                                                  (size_t)J.nsrc * N)) +
               (size_t)l * N * kMomRows * 2;
  // moment k of this source through a resource of its own (size zero for k >= M)
  const double2 *Sm = reinterpret_cast<const double2 *>(J.a);
  const int M = J.nmom;
  const int voff16 = valid ? (int)(i * 16) : 0x7fffffff;
  auto mom_rsrc = [&](int k) { return make_rsrc(Sm + ((size_t)k * J.nsrc + l) * n, k < M ? (int)(n * 16) : 0); };
  double2 acc[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) acc[k] = BufIO<double, 2>::ld(mom_rsrc(k), voff16, 0);
  double2 *p = reinterpret_cast<double2 *>(J.d) + (size_t)l * n;
  const double2 pold = p[ii];
  // shift j's run of this chunk (64 entries of V2<T>, 1 KB apart from the next shift's)
  constexpr int kW = sizeof(V2<T>);
  const int voff = valid ? q * kW : 0x7fffffff;
  const double2 *W = reinterpret_cast<const double2 *>(J.b);
  auto run_rsrc = [&](int j, bool upd) { return make_rsrc(W + blk_chunk(l, c, j, nch, N), upd ? 64 * kW : 0); };
  auto fetch = [&](int j0, double2 (&v)[UB], bool (&f)[UB]) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int j = j0 + u;
      f[u] = j < N && tabi[(size_t)j * kRecI + kUpdI] != 0;
      const V2<T> x = BufIO<T, 2>::ld(run_rsrc(j, f[u]), voff, 0);
      v[u] = make_double2(x.x, x.y);
    }
  };
  double2 nv[UB];
  bool nup[UB];
  if constexpr (PF) fetch(0, nv, nup);
  for (int j0 = 0; j0 < N; j0 += UB) {
    double2 pv[UB];
    bool up[UB];
    if constexpr (PF) {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        pv[u] = nv[u];
        up[u] = nup[u];
      }
      if (j0 + UB < N) fetch(j0 + UB, nv, nup);
    } else {
      fetch(j0, pv, up);
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int j = j0 + u;
      if (up[u]) {  // uniform
        CDbl *gj = gtab + (size_t)j * kMomRows * 2;
        // eight moments at a time: one chunk's coefficients take 32 SGPRs
#pragma unroll
        for (int k0 = 0; k0 < MM; k0 += 8) {
          double gx[8], gy[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            gx[e] = gj[2 * (k0 + e)];
            gy[e] = gj[2 * (k0 + e) + 1];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) cfma(acc[k0 + e], make_double2(gx[e], gy[e]), pv[u]);
        }
      }
      // issued for every shift of the group: the resource of a shift not updated (or
      // past the last) has size zero, and the store moves nothing
      CDbl *t = tabd + (size_t)min(j, N - 1) * kRecD;
      const double2 bj = make_double2(t[2], t[3]), ip = make_double2(t[4], t[5]);
      double2 pn = cmul(ip, rv);
      cfma(pn, bj, pv[u]);
      V2<T> x;
      x.x = pn.x;
      x.y = pn.y;
      BufIO<T, 2>::st(x, run_rsrc(j, up[u]), voff, 0);
    }
  }
#pragma unroll
  for (int k = 0; k < MM; ++k) BufIO<double, 2>::st(acc[k], mom_rsrc(k), voff16, 0);
  if (!valid) return;
  const double beta = S.beta_n;
  double2 pv;
  pv.x = rv.x + beta * pold.x;
  pv.y = rv.y + beta * pold.y;
  p[i] = pv;
}

// ---- block form of the in-loop moment update ----------------------------------
// Over a block of B iterations the seed residuals r(1..B) (r(m) = r_{k0+m}) are kept,
// and every shift direction obeys p_j(s+1) = r(s+1) / pi_j(s) + beta_j(s) p_j(s)
// (Sec. 2.2, with pi_j(s) = pi_{j,k0+s+1}), so
//   p_j(s) = C_j(s) p_j(0) + sum_{m=1..s} D_j(s, m) r(m),
//   C_j(0) = 1, C_j(s+1) = beta_j(s) C_j(s),
//   D_j(s+1, m) = beta_j(s) D_j(s, m) (m <= s), D_j(s+1, s+1) = 1 / pi_j(s).
// The block's moment increments sum_s c_kj alpha_j(s) p_j(s) (eq. 2 summed as the
// solve runs) are then
//   sum_j G_kj p_j(0) + sum_m H_km r(m),
//   G_kj = c_kj A_j,  A_j = sum_s alpha_j(s) C_j(s),
//   H_km = sum_j c_kj E_j(m),  E_j(m) = sum_{s >= m} alpha_j(s) D_j(s, m),
// and p_j(B) follows from the same C and D: one sweep over the entries reads every
// p_j once and writes it once per block instead of once per iteration. A shift not
// updated in an iteration has the identity record (alpha 0, beta 1, 1/pi 0), which
// leaves C, D and the sums unchanged; a source that finished inside the block has
// identity records for the iterations it did not run.

// History records set to the identity, every source fresh, sweep counts to zero.
// nrec = nsrc * nshift * B.
__global__ void blk_init_kernel(ShiftTab *hist, int64_t nrec, unsigned long long *cnt, int32_t *fresh, int nsrc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2 * kBlkCnt) cnt[t] = 0;
  if (t < nsrc) fresh[t] = 1;
  if (t >= nrec) return;
  ShiftTab r;
  r.a = r.ipi = make_double2(0.0, 0.0);
  r.b = make_double2(1.0, 0.0);
  r.upd = r.pad = 0;
  hist[t] = r;
}

// p <- r(s+1) + beta_k p with the beta_k the table kernel staged (the seed direction
// the next dslash reads). job: a = residual ring, d = seed p.
__global__ __launch_bounds__(kBlock) void seed_p_update_kernel(VecBatch B, int slot) {
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int l = lb / J.nblk_vec, vb = lb - l * J.nblk_vec;
  const SeedState &S = J.seed[l];
  if (S.done || !S.pending || S.brk_n) return;  // uniform over the block
  const double beta = S.beta_n;
  const double2 *r = reinterpret_cast<const double2 *>(J.a) + ((size_t)slot * J.nsrc + l) * J.n;
  double2 *p = reinterpret_cast<double2 *>(J.d) + (size_t)l * J.n;
  const int64_t stride = (int64_t)J.nblk_vec * kBlock * kEpt;
  for (int64_t base = (int64_t)vb * kBlock * kEpt + threadIdx.x; base - threadIdx.x < J.n; base += stride) {
    double2 rv[kEpt], pv[kEpt];
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < J.n) {  // streaming: neither vector is re-read before it leaves the caches
        rv[e] = ldc<true>(r + i);
        pv[e] = ldc<true>(p + i);
      }
    }
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < J.n) stc<true>(p + i, make_double2(rv[e].x + beta * pv[e].x, rv[e].y + beta * pv[e].y));
    }
  }
}

// Composition of a block's records, one block of threads per source: a thread per
// shift runs the recurrences of C_j, D_j, A_j and E_j over the B records (and resets
// them), writes C_j, the flags, D_j and G_kj, and leaves E_j in the work area; after a
// barrier the threads form H_km = sum_j c_kj E_j(m). A record with upd = 0 is skipped
// (it is the identity). job: e = table.
template <int BB>
__global__ __launch_bounds__(kBlock) void blk_compose_kernel(VecBatch B, int prec) {
  __shared__ int n_any, n_st;
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int l = b - J.block_begin;
  const int N = J.nshift;
  const BlkLayout lay = blk_layout(J.nsrc, N, BB);
  char *tb = reinterpret_cast<char *>(J.e);
  ShiftTab *hist = reinterpret_cast<ShiftTab *>(tb + lay.hist) + (size_t)l * N * BB;
  double2 *g = reinterpret_cast<double2 *>(tb + lay.g) + (size_t)l * N * kMomRows;
  BlkShift *cs = reinterpret_cast<BlkShift *>(tb + lay.comp) + (size_t)l * N;
  double2 *D = reinterpret_cast<double2 *>(tb + lay.d) + (size_t)l * N * BB;
  double2 *H = reinterpret_cast<double2 *>(tb + lay.h) + (size_t)l * kMomRows * BB;
  double2 *E = reinterpret_cast<double2 *>(tb + lay.e) + (size_t)l * N * BB;
  int32_t *anyf = reinterpret_cast<int32_t *>(tb + lay.any);
  if (threadIdx.x == 0) n_any = n_st = 0;
  __syncthreads();
  const double2 zero = make_double2(0.0, 0.0);
  int any_t = 0, st_t = 0;
  for (int j = threadIdx.x; j < N; j += kBlock) {
    // C_j and A_j in registers; the rows D_j(s, .) and E_j(.) are updated in place in
    // the table (row m - 1 for m = 1..BB: a few L2-resident kilobytes per shift)
    double2 C = make_double2(1.0, 0.0), A = zero;
    double2 *d = D + (size_t)j * BB, *e = E + (size_t)j * BB;
    for (int m = 0; m < BB; ++m) d[m] = e[m] = zero;
    int any = 0, frz = 0;
    ShiftTab *h = hist + (size_t)j * BB;
    for (int s = 0; s < BB; ++s) {
      const ShiftTab t = h[s];
      if (t.upd) {  // a record not updated is the identity
        cfma(A, t.a, C);
        for (int m = 0; m < s; ++m) {
          const double2 dm = d[m];
          cfma(e[m], t.a, dm);
          d[m] = cmul(t.b, dm);
        }
        C = cmul(t.b, C);
        d[s] = t.ipi;
      }
      any |= t.upd;
      frz |= t.pad;
    }
    ShiftTab idr;
    idr.a = idr.ipi = zero;
    idr.b = make_double2(1.0, 0.0);
    idr.upd = idr.pad = 0;
    for (int s = 0; s < BB; ++s) h[s] = idr;
    BlkShift o;
    o.c = C;
    o.any = any;
    o.st = any && !frz;
    o.pad[0] = o.pad[1] = 0;
    cs[j] = o;
    for (int k = 0; k < kMomRows; ++k)
      g[(size_t)j * kMomRows + k] = (any && k < J.nmom) ? cmul(J.mcoef[(size_t)k * N + j], A) : zero;
    any_t += any;
    st_t += o.st;
  }
  if (any_t) atomicAdd(&n_any, any_t);
  if (st_t) atomicAdd(&n_st, st_t);
  __syncthreads();  // (also orders this block's E writes before the reads below)
  for (int t = threadIdx.x; t < kMomRows * BB; t += kBlock) {
    const int k = t / BB, m = t - k * BB;
    double2 acc = zero;
    if (k < J.nmom)
      for (int j = 0; j < N; ++j) cfma(acc, J.mcoef[(size_t)k * N + j], E[(size_t)j * BB + m]);
    H[t] = acc;
  }
  if (threadIdx.x == 0) {
    // the source's first block: its directions were never written (every p_j(0) = v)
    int32_t *fresh = reinterpret_cast<int32_t *>(tb + lay.fresh) + l;
    const int first = *fresh != 0 && n_any > 0;
    if (first) *fresh = 0;
    anyf[l] = (n_any > 0 ? 1 : 0) | (n_st > 0 ? 2 : 0) | (first ? 4 : 0);
    // what the two sweep kernels will move for this source (moment kernel: runs if a
    // shift moved, reads those directions; direction kernel: runs if a shift is still
    // active, reads the moved directions, writes the active ones)
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(tb + lay.cnt) + prec * kBlkCnt;
    // (a first block reads v once instead of its directions: counted as one FP64
    // direction read, in the FP64 counts it always falls in)
    const unsigned long long nrd = first ? 1 : (unsigned long long)n_any;
    unsigned long long *crd = first ? reinterpret_cast<unsigned long long *>(tb + lay.cnt) : cnt;
    if (n_any > 0) {
      atomicAdd(cnt + 0, 1ull);
      atomicAdd(crd + 1, nrd);
    }
    if (n_st > 0) {
      atomicAdd(cnt + 2, 1ull);
      atomicAdd(crd + 3, nrd);
      atomicAdd(cnt + 4, (unsigned long long)n_st);
    }
  }
}

// The block's sweep, in two kernels over the in-loop kernel's grid (one thread per
// entry of one source, chunk-blocked directions) that never hold the moment sums and
// the block's residuals at the same time, so both run with few registers and many
// wavefronts per SIMD: the moment kernel reads every p_j(0) and the residuals and
// adds sum_j G_kj p_j(0) + sum_m H_km r(m) to the MM moment sums; the direction kernel
// then reads every p_j(0) again and writes p_j(B) = C_j p_j(0) + sum_m D_j(B, m) r(m)
// for the shifts still active. The coefficients are read at wavefront-uniform
// addresses through the constant address space (scalar loads). Each kernel keeps PD
// directions in flight per thread: shift j's direction is loaded PD shifts ahead into
// buffer slot j mod PD, in groups of PD shifts (a static slot per unrolled step, so no
// register is copied while its load is in flight), the first group peeled so the loop
// is entered with the memory operations in flight that every later group starts with.
// A source's first block reads v (job d) in place of every p_j(0): the directions are
// not initialised at the start of a solve.
// job: a = moments, b = shift directions, c = residual ring, d = sources v, e = table.
struct BlkView {
  typedef __attribute__((address_space(4))) const double CDbl;
  typedef __attribute__((address_space(4))) const int32_t CInt;
  static constexpr int kCsD = sizeof(BlkShift) / sizeof(double), kCsI = sizeof(BlkShift) / sizeof(int32_t);
  static constexpr int kAnyI = offsetof(BlkShift, any) / sizeof(int32_t);
  static constexpr int kStI = offsetof(BlkShift, st) / sizeof(int32_t);
  CInt *anyf, *csi;
  CDbl *csd, *Dt, *gtab, *Ht;
  __device__ BlkView(const VecJob &J, int l, int BB) {
    const BlkLayout lay = blk_layout(J.nsrc, J.nshift, BB);
    const uintptr_t tb = reinterpret_cast<uintptr_t>(J.e);
    const int N = J.nshift;
    anyf = reinterpret_cast<CInt *>(tb + lay.any);
    csd = reinterpret_cast<CDbl *>(tb + lay.comp) + (size_t)l * N * kCsD;
    csi = reinterpret_cast<CInt *>(tb + lay.comp) + (size_t)l * N * kCsI;
    Dt = reinterpret_cast<CDbl *>(tb + lay.d) + (size_t)l * N * BB * 2;
    gtab = reinterpret_cast<CDbl *>(tb + lay.g) + (size_t)l * N * kMomRows * 2;
    Ht = reinterpret_cast<CDbl *>(tb + lay.h) + (size_t)l * kMomRows * BB * 2;
  }
  __device__ bool any(int j) const { return csi[(size_t)j * kCsI + kAnyI] != 0; }
  __device__ bool st(int j) const { return csi[(size_t)j * kCsI + kStI] != 0; }
};

// Thread geometry of the sweep kernels.
struct BlkLane {
  int l;          // source
  int64_t i;      // entry
  bool valid;     // i < n
  int64_t ii;     // entry read by the thread (0 for invalid lanes, which store nothing)
  int64_t c;      // chunk of the wavefront
  int q;          // place in the chunk
  __device__ BlkLane(const VecJob &J, int lb) {
    l = lb / J.nblk_mom;
    const int vb = lb - l * J.nblk_mom;
    i = (int64_t)vb * kMomBlock + threadIdx.x;
    valid = i < J.n;
    ii = valid ? i : 0;
    c = (int64_t)vb * (kMomBlock / 64) + uni(threadIdx.x >> 6);  // i >> 6, in a scalar register
    q = (int)(i & 63);
  }
};

template <typename T, int MM, int BB, int PD>
__global__ __launch_bounds__(kMomBlock) void blk_moments_kernel(VecBatch B) {
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const BlkLane t(J, b - J.block_begin);
  const int l = t.l, N = J.nshift;
  const BlkView v(J, l, BB);
  if ((v.anyf[l] & 1) == 0) return;  // no shift of the source moved in the block
  const int64_t n = J.n, nch = (n + 63) / 64;
  const double2 *Sm = reinterpret_cast<const double2 *>(J.a);
  const int M = J.nmom;
  const int voff16 = t.valid ? (int)(t.i * 16) : 0x7fffffff;
  auto mom_rsrc = [&](int k) { return make_rsrc(Sm + ((size_t)k * J.nsrc + l) * n, k < M ? (int)(n * 16) : 0); };
  double2 acc[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) acc[k] = BufIO<double, 2>::ld(mom_rsrc(k), voff16, 0);
  // a source's first block: every p_j(0) is v (the directions were never written)
  const bool fresh = (v.anyf[l] & 4) != 0;
  const double2 v0 = reinterpret_cast<const double2 *>(J.d)[(size_t)l * n + t.ii];
  constexpr int kW = sizeof(V2<T>);
  const int voff = t.valid ? t.q * kW : 0x7fffffff;
  const double2 *W = reinterpret_cast<const double2 *>(J.b);
  auto fetch = [&](int j, double2 &x, bool &f) {
    f = j < N && v.any(j);
    const V2<T> y =
        BufIO<T, 2>::ld(make_rsrc(W + blk_chunk(l, t.c, j, nch, N), f && !fresh ? 64 * kW : 0), voff, 0);
    x = fresh ? v0 : make_double2(y.x, y.y);
  };
  double2 buf[PD];
  bool bup[PD];
#pragma unroll
  for (int u = 0; u < PD; ++u) fetch(u, buf[u], bup[u]);
  auto group = [&](int j0) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int j = j0 + u;
      const double2 pv = buf[u];
      if (bup[u]) {  // uniform
        BlkView::CDbl *gj = v.gtab + (size_t)j * kMomRows * 2;
#pragma unroll
        for (int k0 = 0; k0 < MM; k0 += 8) {
          double gx[8], gy[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            gx[e] = gj[2 * (k0 + e)];
            gy[e] = gj[2 * (k0 + e) + 1];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) cfma(acc[k0 + e], make_double2(gx[e], gy[e]), pv);
        }
      }
      fetch(j + PD, buf[u], bup[u]);
      // keeps the refill here (the scheduler would otherwise gather the group's loads
      // at its end, leaving none in flight while the next group starts)
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  group(0);
  for (int j0 = PD; j0 < N; j0 += PD) group(j0);
  // residual terms, one residual at a time
  const double2 *ring = reinterpret_cast<const double2 *>(J.c);
  for (int m = 0; m < BB; ++m) {
    const double2 r = ldc<true>(ring + ((size_t)m * J.nsrc + l) * n + t.ii);
    BlkView::CDbl *hm = v.Ht + 2 * m;
#pragma unroll
    for (int k = 0; k < MM; ++k) cfma(acc[k], make_double2(hm[2 * BB * k], hm[2 * BB * k + 1]), r);
  }
#pragma unroll
  for (int k = 0; k < MM; ++k) BufIO<double, 2>::st(acc[k], mom_rsrc(k), voff16, 0);
}

template <typename T, int BB, int PD>
__global__ __launch_bounds__(kMomBlock) void blk_dirs_kernel(VecBatch B) {
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const BlkLane t(J, b - J.block_begin);
  const int l = t.l, N = J.nshift;
  const BlkView v(J, l, BB);
  if ((v.anyf[l] & 2) == 0) return;  // every shift of the source froze (or none moved)
  const int64_t n = J.n, nch = (n + 63) / 64;
  const double2 *ring = reinterpret_cast<const double2 *>(J.c);
  double2 rv[BB];
#pragma unroll
  for (int m = 0; m < BB; ++m) rv[m] = ldc<true>(ring + ((size_t)m * J.nsrc + l) * n + t.ii);
  constexpr int kW = sizeof(V2<T>);
  const int voff = t.valid ? t.q * kW : 0x7fffffff;
  const double2 *W = reinterpret_cast<const double2 *>(J.b);
  auto run_rsrc = [&](int j, bool on) { return make_rsrc(W + blk_chunk(l, t.c, j, nch, N), on ? 64 * kW : 0); };
  const bool fresh = (v.anyf[l] & 4) != 0;  // a source's first block: every p_j(0) is v
  const double2 v0 = reinterpret_cast<const double2 *>(J.d)[(size_t)l * n + t.ii];
  auto fetch = [&](int j, double2 &x, bool &f) {
    f = j < N && v.any(j);
    const V2<T> y = BufIO<T, 2>::ld(run_rsrc(j, f && !fresh), voff, 0);
    x = fresh ? v0 : make_double2(y.x, y.y);
  };
  double2 buf[PD];
  bool bup[PD];
#pragma unroll
  for (int u = 0; u < PD; ++u) fetch(u, buf[u], bup[u]);
  auto group = [&](int j0) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int j = j0 + u;
      const int jj = min(j, N - 1);  // coefficients of a shift past the last are not used
      const double2 pv = buf[u];
      const bool stj = bup[u] && v.st(jj);
      BlkView::CDbl *cj = v.csd + (size_t)jj * BlkView::kCsD;
      BlkView::CDbl *dj = v.Dt + (size_t)jj * BB * 2;
      double2 pn = cmul(make_double2(cj[0], cj[1]), pv);
#pragma unroll
      for (int m = 0; m < BB; ++m) cfma(pn, make_double2(dj[2 * m], dj[2 * m + 1]), rv[m]);
      V2<T> x;
      x.x = pn.x;
      x.y = pn.y;
      BufIO<T, 2>::st(x, run_rsrc(jj, stj), voff, 0);
      fetch(j + PD, buf[u], bup[u]);
    }
  };
  group(0);
  for (int j0 = PD; j0 < N; j0 += PD) group(j0);
}

// Start of an in-loop solve: p_j = v_l in the chunk-blocked layout (padding zero).
// Grid: (ceil(nch 64 / kBlock), nsrc * nshift).
__global__ void init_shifts_blocked_kernel(double2 *W, const double2 *v, int64_t n, int nshift) {
  const int slot = blockIdx.y;
  const int l = slot / nshift, j = slot - l * nshift;
  const int64_t nch = (n + 63) / 64;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nch * 64) return;
  W[blk_chunk(l, i >> 6, j, nch, nshift) + (i & 63)] = i < n ? v[(size_t)l * n + i] : make_double2(0.0, 0.0);
}

// FP32 switch of the chunk-blocked directions, in place: one wavefront per (source,
// chunk, shift) run reads its 64 double2 and writes them back as 64 float2 into the
// run's first half (the store depends on the loaded values, so the whole run is read
// before any of it is written). nruns = nsrc * nch * nshift.
__global__ void blocked_to_fp32_kernel(double2 *W, int64_t nruns) {
  const int64_t run = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (run >= nruns) return;
  const int q = threadIdx.x & 63;
  double2 *base = W + (size_t)run * 64;
  const double2 x = base[q];
  reinterpret_cast<float2 *>(base)[q] = make_float2((float)x.x, (float)x.y);
}

// Reliable update: r64 = r_base - B x_part (q = B x_part already computed in FP64),
// r32 = (float) r64, partial <r64, r64>. job: a = r_base, b = q64, c = r64, d = r32.
__global__ __launch_bounds__(kBlock) void reliable_residual_kernel(VecBatch B) {
  __shared__ double red[kBlock / 64];
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int l = lb / J.nblk_vec, vb = lb - l * J.nblk_vec;
  if (J.seed[l].done) return;
  const size_t off = (size_t)l * J.n;
  const double2 *rb = reinterpret_cast<const double2 *>(J.a) + off;
  const double2 *q = reinterpret_cast<const double2 *>(J.b) + off;
  double2 *r64 = reinterpret_cast<double2 *>(J.c) + off;
  float2 *r32 = reinterpret_cast<float2 *>(J.d) + off;
  double acc = 0.0;
  const int64_t stride = (int64_t)J.nblk_vec * kBlock * kEpt;
  for (int64_t base = (int64_t)vb * kBlock * kEpt + threadIdx.x; base - threadIdx.x < J.n; base += stride) {
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < J.n) {
        const double2 rv = rb[i] - q[i];
        r64[i] = rv;
        r32[i] = make_float2((float)rv.x, (float)rv.y);
        acc += rv.x * rv.x + rv.y * rv.y;
      }
    }
  }
  const double tot = block_sum_all<kBlock / 64>(acc, red);
  if (threadIdx.x == 0) J.partial[(size_t)l * J.nblk_vec + vb] = tot;
}

// x_part64 += x_part32, x_part32 = 0. job: a = x_part64, b = x_part32.
__global__ __launch_bounds__(kBlock) void fold_seed_kernel(VecBatch B) {
  const int b = blockIdx.x;
  const VecJob &J = B.job[job_of(B.job, B.njobs, b)];
  const int lb = b - J.block_begin;
  const int l = lb / J.nblk_vec, vb = lb - l * J.nblk_vec;
  if (J.seed[l].done) return;
  const size_t off = (size_t)l * J.n;
  double2 *x64 = reinterpret_cast<double2 *>(J.a) + off;
  float2 *x32 = reinterpret_cast<float2 *>(J.b) + off;
  const int64_t stride = (int64_t)J.nblk_vec * kBlock * kEpt;
  for (int64_t base = (int64_t)vb * kBlock * kEpt + threadIdx.x; base - threadIdx.x < J.n; base += stride) {
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const int64_t i = base + (int64_t)e * kBlock;
      if (i < J.n) {
        const float2 xv = x32[i];
        double2 xm = x64[i];
        xm.x += (double)xv.x;
        xm.y += (double)xv.y;
        x64[i] = xm;
        x32[i] = make_float2(0.f, 0.f);
      }
    }
  }
}

// Start of a solve: p_j = v_l and x_j = 0 for every (source, shift) slot.
__global__ void init_shifts_kernel(double2 *y, double2 *W, const double2 *v, int64_t n, int nshift) {
  const size_t slot = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t l = slot / nshift;
  W[slot * n + i] = v[l * n + i];
  if (y) y[slot * n + i] = make_double2(0.0, 0.0);
}

// End of an FP32 phase: x_j += x_part_j, x_part_j = 0 for every (source, shift)
// slot; the FP32 partial is the upper half of the slot's workspace.
__global__ void fold_shifts_kernel(double2 *y, double2 *W, int64_t n) {
  const size_t slot = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 *x32 = reinterpret_cast<float2 *>(W + slot * n) + n;
  double2 *ys = y + slot * n;
  const float2 xv = x32[i];
  double2 v = ys[i];
  v.x += (double)xv.x;
  v.y += (double)xv.y;
  ys[i] = v;
  x32[i] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// Plain conversions and reductions over flat complex arrays.
__global__ void to_fp32_kernel(const double2 *src, float2 *dst, float2 *zero, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
    if (zero) zero[i] = make_float2(0.f, 0.f);
  }
}

template <typename S, typename D>
__global__ void cast_kernel(const S *src, D *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const S v = src[i];
    D d;
    d.x = v.x;
    d.y = v.y;
    dst[i] = d;
  }
}

// canonical complex128 [nsrc][V][12] -> planar T [nsrc][12][V]; thread per (src, c, s)
template <typename T>
__global__ void pack_kernel(const double2 *canon, V2<T> *planar, int nsrc, int V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nsrc * 12 * V;
  if (i >= tot) return;
  const int64_t l = i / (12 * (int64_t)V);
  const int64_t rem = i - l * 12 * V;
  const int c = (int)(rem / V);
  const int s = (int)(rem - (int64_t)c * V);
  const double2 v = canon[(l * V + s) * 12 + c];
  V2<T> o;
  o.x = (T)v.x;
  o.y = (T)v.y;
  planar[i] = o;
}
template <typename T>
__global__ void unpack_kernel(const V2<T> *planar, double2 *canon, int nsrc, int V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nsrc * 12 * V;
  if (i >= tot) return;
  const int64_t l = i / (12 * (int64_t)V);
  const int64_t rem = i - l * 12 * V;
  const int s = (int)(rem / 12);
  const int c = (int)(rem - (int64_t)s * 12);
  const V2<T> v = planar[(l * 12 + c) * V + s];
  canon[i] = make_double2((double)v.x, (double)v.y);
}

// partial[v][blk] = sum over the block's entries of |x_v|^2 (nvec vectors of n)
__global__ __launch_bounds__(kBlock) void norm2_kernel(const double2 *x, int64_t n, double *partial, int nblk) {
  __shared__ double red[kBlock / 64];
  const int vec = blockIdx.y;
  const double2 *xv = x + (size_t)vec * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)nblk * kBlock) {
    const double2 v = xv[i];
    acc += v.x * v.x + v.y * v.y;
  }
  const double tot = block_sum_all<kBlock / 64>(acc, red);
  if (threadIdx.x == 0) partial[(size_t)vec * nblk + blockIdx.x] = tot;
}

// partial of || v - z_j y_j + (A y_j) ||^2 for nvec shifts of one source
__global__ __launch_bounds__(kBlock) void true_residual_kernel(const double2 *v, const double2 *y,
                                                               const double2 *Ay, const double *z,
                                                               int64_t n, double *partial, int nblk) {
  __shared__ double red[kBlock / 64];
  const int j = blockIdx.y;
  const double2 zj = make_double2(z[2 * j], z[2 * j + 1]);
  const double2 *yj = y + (size_t)j * n;
  const double2 *ayj = Ay + (size_t)j * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)nblk * kBlock) {
    const double2 zy = cmul(zj, yj[i]);
    const double2 rv = v[i] - zy + ayj[i];
    acc += rv.x * rv.x + rv.y * rv.y;
  }
  const double tot = block_sum_all<kBlock / 64>(acc, red);
  if (threadIdx.x == 0) partial[(size_t)j * nblk + blockIdx.x] = tot;
}

// s_{l,k} = sum_j c[k][j] y_{l,j}; grid (entry blocks, source, moment chunk)
constexpr int kMomChunk = 8;
__global__ __launch_bounds__(kBlock) void moments_kernel(const double2 *y, int nshift, int64_t y_stride_l,
                                                         const double2 *c, int nmom, double2 *s, int64_t n,
                                                         int64_t s_stride_l, int64_t s_stride_k) {
  extern __shared__ double2 csh[];  // [kMomChunk][nshift]
  const int l = blockIdx.y;
  const int k0 = blockIdx.z * kMomChunk;
  const int nk = min(kMomChunk, nmom - k0);
  for (int t = threadIdx.x; t < nk * nshift; t += kBlock) {
    const int kk = t / nshift, j = t - kk * nshift;
    csh[t] = c[(size_t)(k0 + kk) * nshift + j];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double2 acc[kMomChunk];
#pragma unroll
  for (int kk = 0; kk < kMomChunk; ++kk) acc[kk] = make_double2(0, 0);
  const double2 *yl = y + (size_t)l * y_stride_l * n;
  for (int j = 0; j < nshift; ++j) {
    const double2 yv = yl[(size_t)j * n + i];
#pragma unroll
    for (int kk = 0; kk < kMomChunk; ++kk)
      if (kk < nk) cfma(acc[kk], csh[kk * nshift + j], yv);
  }
#pragma unroll
  for (int kk = 0; kk < kMomChunk; ++kk)
    if (kk < nk) s[((size_t)l * s_stride_l + (size_t)(k0 + kk) * s_stride_k) * n + i] = acc[kk];
}

// ---------------------------------------------------------------------------
void launch_seed_alpha(const ScalarBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(seed_alpha_kernel, dim3(b.total_blocks), dim3(kBlock), 0, st, b);
}
void launch_commit(const DslashBatch &b, hipStream_t st) {
  if (b.njobs <= 0) return;
  hipLaunchKernelGGL(commit_kernel, dim3(b.njobs), dim3(kBlock), 0, st, b);
}
void launch_seed_r_update(const VecBatch &b, int prec, hipStream_t st, int slot) {
  if (prec == 0) hipLaunchKernelGGL(seed_r_update_kernel<double>, dim3(b.total_blocks), dim3(kBlock), 0, st, b, slot);
  else hipLaunchKernelGGL(seed_r_update_kernel<float>, dim3(b.total_blocks), dim3(kBlock), 0, st, b, slot);
}
template <typename T, typename TR, bool FOLD, int U>
static void launch_su_nt(const VecBatch &b, int nt, hipStream_t st) {
  if (nt) hipLaunchKernelGGL((shift_update_kernel<T, TR, FOLD, U, true>), dim3(b.total_blocks), dim3(kBlock), 0, st, b);
  else hipLaunchKernelGGL((shift_update_kernel<T, TR, FOLD, U, false>), dim3(b.total_blocks), dim3(kBlock), 0, st, b);
}
template <typename T, typename TR, bool FOLD>
static void launch_su_u(const VecBatch &b, int unroll, int nt, hipStream_t st) {
  if (unroll >= 4) launch_su_nt<T, TR, FOLD, 4>(b, nt, st);
  else if (unroll == 2) launch_su_nt<T, TR, FOLD, 2>(b, nt, st);
  else launch_su_nt<T, TR, FOLD, 1>(b, nt, st);
}
void launch_shift_update(const VecBatch &b, int prec, int seed_prec, int fold, int unroll, int nt, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  if (prec == 0) launch_su_u<double, double, false>(b, unroll, nt, st);
  else if (seed_prec == 0) {
    if (fold) launch_su_u<float, double, true>(b, unroll, nt, st);
    else launch_su_u<float, double, false>(b, unroll, nt, st);
  } else {
    if (fold) launch_su_u<float, float, true>(b, unroll, nt, st);
    else launch_su_u<float, float, false>(b, unroll, nt, st);
  }
}
void launch_shift_table(const VecBatch &b, hipStream_t st, int slot) {
  if (b.total_blocks <= 0) return;
  hipLaunchKernelGGL(shift_table_kernel, dim3(b.total_blocks), dim3(kBlock), 0, st, b, slot);
}
template <typename T, int MM>
static void launch_smt_ub(const VecBatch &b, int ub, int pf, hipStream_t st) {
  const dim3 g(b.total_blocks), t(kMomBlock);
  if (pf) {
    if (ub >= 2) hipLaunchKernelGGL((shift_moments_tab_kernel<T, MM, 2, 1>), g, t, 0, st, b);
    else hipLaunchKernelGGL((shift_moments_tab_kernel<T, MM, 1, 1>), g, t, 0, st, b);
    return;
  }
  if (ub >= 4) hipLaunchKernelGGL((shift_moments_tab_kernel<T, MM, 4, 0>), g, t, 0, st, b);
  else if (ub == 2) hipLaunchKernelGGL((shift_moments_tab_kernel<T, MM, 2, 0>), g, t, 0, st, b);
  else hipLaunchKernelGGL((shift_moments_tab_kernel<T, MM, 1, 0>), g, t, 0, st, b);
}
template <typename T>
static void launch_smt(const VecBatch &b, int mm, int ub, int pf, hipStream_t st) {
  if (mm <= 8) launch_smt_ub<T, 8>(b, ub, pf, st);
  else if (mm <= 16) launch_smt_ub<T, 16>(b, ub, pf, st);
  else if (mm <= 24) launch_smt_ub<T, 24>(b, ub, pf, st);
  else launch_smt_ub<T, 32>(b, ub, pf, st);
}
void launch_shift_moments_tab(const VecBatch &b, int prec, int nmom_max, int ub, int pf, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  if (prec == 0) launch_smt<double>(b, nmom_max, ub, pf, st);
  else launch_smt<float>(b, nmom_max, ub, pf, st);
}
void launch_reliable_residual(const VecBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(reliable_residual_kernel, dim3(b.total_blocks), dim3(kBlock), 0, st, b);
}
void launch_fold_seed(const VecBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(fold_seed_kernel, dim3(b.total_blocks), dim3(kBlock), 0, st, b);
}
static inline unsigned nblocks1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
void launch_to_fp32(const void *src64, void *dst32, void *zero32, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_fp32_kernel, dim3(nblocks1d(n)), dim3(kBlock), 0, st,
                     (const double2 *)src64, (float2 *)dst32, (float2 *)zero32, n);
}
void launch_blk_init(void *tab, int nsrc, int nshift, int B, hipStream_t st) {
  const int64_t nrec = (int64_t)nsrc * nshift * B;
  if (nrec <= 0) return;
  const BlkLayout lay = blk_layout(nsrc, nshift, B);
  char *tb = reinterpret_cast<char *>(tab);
  hipLaunchKernelGGL(blk_init_kernel, dim3(nblocks1d(std::max<int64_t>({nrec, 2 * kBlkCnt, nsrc}))), dim3(kBlock),
                     0, st, reinterpret_cast<ShiftTab *>(tb + lay.hist), nrec,
                     reinterpret_cast<unsigned long long *>(tb + lay.cnt), reinterpret_cast<int32_t *>(tb + lay.fresh),
                     nsrc);
}
void launch_seed_p_update(const VecBatch &b, int slot, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  hipLaunchKernelGGL(seed_p_update_kernel, dim3(b.total_blocks), dim3(kBlock), 0, st, b, slot);
}
void launch_blk_compose(const VecBatch &b, int B, int prec, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  const dim3 g(b.total_blocks), t(kBlock);
  const int ph = prec == 0 ? 0 : 1;
  if (B == 4) hipLaunchKernelGGL(blk_compose_kernel<4>, g, t, 0, st, b, ph);
  else if (B == 8) hipLaunchKernelGGL(blk_compose_kernel<8>, g, t, 0, st, b, ph);
  else if (B == 16) hipLaunchKernelGGL(blk_compose_kernel<16>, g, t, 0, st, b, ph);
  else if (B == 24) hipLaunchKernelGGL(blk_compose_kernel<24>, g, t, 0, st, b, ph);
  else hipLaunchKernelGGL(blk_compose_kernel<32>, g, t, 0, st, b, ph);
}
constexpr int kBlkPD = 4;  // shift directions in flight per thread of the sweep kernels
template <typename T, int MM>
static void launch_bm(const VecBatch &b, int B, hipStream_t st) {
  const dim3 g(b.total_blocks), t(kMomBlock);
  if (B == 4) hipLaunchKernelGGL((blk_moments_kernel<T, MM, 4, kBlkPD>), g, t, 0, st, b);
  else if (B == 8) hipLaunchKernelGGL((blk_moments_kernel<T, MM, 8, kBlkPD>), g, t, 0, st, b);
  else if (B == 16) hipLaunchKernelGGL((blk_moments_kernel<T, MM, 16, kBlkPD>), g, t, 0, st, b);
  else if (B == 24) hipLaunchKernelGGL((blk_moments_kernel<T, MM, 24, kBlkPD>), g, t, 0, st, b);
  else hipLaunchKernelGGL((blk_moments_kernel<T, MM, 32, kBlkPD>), g, t, 0, st, b);
}
template <typename T>
static void launch_bd(const VecBatch &b, int B, hipStream_t st) {
  const dim3 g(b.total_blocks), t(kMomBlock);
  if (B == 4) hipLaunchKernelGGL((blk_dirs_kernel<T, 4, kBlkPD>), g, t, 0, st, b);
  else if (B == 8) hipLaunchKernelGGL((blk_dirs_kernel<T, 8, kBlkPD>), g, t, 0, st, b);
  else if (B == 16) hipLaunchKernelGGL((blk_dirs_kernel<T, 16, kBlkPD>), g, t, 0, st, b);
  else if (B == 24) hipLaunchKernelGGL((blk_dirs_kernel<T, 24, kBlkPD>), g, t, 0, st, b);
  else hipLaunchKernelGGL((blk_dirs_kernel<T, 32, kBlkPD>), g, t, 0, st, b);
}
template <typename T>
static void launch_bp(const VecBatch &b, int mm, int B, hipStream_t st) {
  if (mm <= 8) launch_bm<T, 8>(b, B, st);
  else if (mm <= 16) launch_bm<T, 16>(b, B, st);
  else if (mm <= 24) launch_bm<T, 24>(b, B, st);
  else launch_bm<T, 32>(b, B, st);
  launch_bd<T>(b, B, st);
}
void launch_blk_pass(const VecBatch &b, int prec, int nmom_max, int B, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  if (prec == 0) launch_bp<double>(b, nmom_max, B, st);
  else launch_bp<float>(b, nmom_max, B, st);
}
void launch_init_shifts_blocked(void *W, const void *v, int64_t n, int nsrc, int nshift, hipStream_t st) {
  const int64_t npad = (n + 63) / 64 * 64;
  hipLaunchKernelGGL(init_shifts_blocked_kernel, dim3(nblocks1d(npad), nsrc * nshift), dim3(kBlock), 0, st,
                     (double2 *)W, (const double2 *)v, n, nshift);
}
void launch_blocked_to_fp32(void *W, int64_t n, int nsrc, int nshift, hipStream_t st) {
  const int64_t nruns = (int64_t)nsrc * ((n + 63) / 64) * nshift;
  const int64_t per = kBlock / 64;
  hipLaunchKernelGGL(blocked_to_fp32_kernel, dim3((unsigned)((nruns + per - 1) / per)), dim3(kBlock), 0, st,
                     (double2 *)W, nruns);
}
void launch_init_shifts(void *y, void *W, const void *v, int64_t n, int nsrc, int nshift, hipStream_t st) {
  if (n <= 0 || nsrc * nshift <= 0) return;
  hipLaunchKernelGGL(init_shifts_kernel, dim3(nblocks1d(n), nsrc * nshift), dim3(kBlock), 0, st, (double2 *)y,
                     (double2 *)W, (const double2 *)v, n, nshift);
}
void launch_fold_shifts(void *y, void *W, int64_t n, int nslots, hipStream_t st) {
  if (n <= 0 || nslots <= 0) return;
  hipLaunchKernelGGL(fold_shifts_kernel, dim3(nblocks1d(n), nslots), dim3(kBlock), 0, st, (double2 *)y,
                     (double2 *)W, n);
}
void launch_cast(const void *src, int sp, void *dst, int dp, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  if (sp == 0 && dp == 1)
    hipLaunchKernelGGL((cast_kernel<double2, float2>), dim3(nblocks1d(n)), dim3(kBlock), 0, st, (const double2 *)src, (float2 *)dst, n);
  else if (sp == 1 && dp == 0)
    hipLaunchKernelGGL((cast_kernel<float2, double2>), dim3(nblocks1d(n)), dim3(kBlock), 0, st, (const float2 *)src, (double2 *)dst, n);
  else if (sp == 0)
    hipLaunchKernelGGL((cast_kernel<double2, double2>), dim3(nblocks1d(n)), dim3(kBlock), 0, st, (const double2 *)src, (double2 *)dst, n);
  else
    hipLaunchKernelGGL((cast_kernel<float2, float2>), dim3(nblocks1d(n)), dim3(kBlock), 0, st, (const float2 *)src, (float2 *)dst, n);
}
void launch_pack(const void *canon, void *planar, int prec, int nsrc, int V, hipStream_t st) {
  const int64_t tot = (int64_t)nsrc * 12 * V;
  if (tot <= 0) return;
  if (prec == 0) hipLaunchKernelGGL(pack_kernel<double>, dim3(nblocks1d(tot)), dim3(kBlock), 0, st, (const double2 *)canon, (double2 *)planar, nsrc, V);
  else hipLaunchKernelGGL(pack_kernel<float>, dim3(nblocks1d(tot)), dim3(kBlock), 0, st, (const double2 *)canon, (float2 *)planar, nsrc, V);
}
void launch_unpack(const void *planar, int prec, void *canon, int nsrc, int V, hipStream_t st) {
  const int64_t tot = (int64_t)nsrc * 12 * V;
  if (tot <= 0) return;
  if (prec == 0) hipLaunchKernelGGL(unpack_kernel<double>, dim3(nblocks1d(tot)), dim3(kBlock), 0, st, (const double2 *)planar, (double2 *)canon, nsrc, V);
  else hipLaunchKernelGGL(unpack_kernel<float>, dim3(nblocks1d(tot)), dim3(kBlock), 0, st, (const float2 *)planar, (double2 *)canon, nsrc, V);
}
void launch_norm2_partial(const void *x, int64_t n, int nvec, double *partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(norm2_kernel, dim3(nblk, nvec), dim3(kBlock), 0, st, (const double2 *)x, n, partial, nblk);
}
void launch_true_residual(const void *v, const void *y, const void *Ay, const double *z, int64_t n,
                          int nvec, double *partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(true_residual_kernel, dim3(nblk, nvec), dim3(kBlock), 0, st, (const double2 *)v,
                     (const double2 *)y, (const double2 *)Ay, z, n, partial, nblk);
}
void launch_moments_strided2(const void *y, int nsrc, int nshift, int64_t y_stride_l, const double *c_dev, int nmom,
                             void *s, int64_t n, int64_t sl, int64_t sk, hipStream_t st) {
  const dim3 grid(nblocks1d(n), nsrc, (nmom + kMomChunk - 1) / kMomChunk);
  const size_t shm = (size_t)kMomChunk * nshift * sizeof(double2);
  hipLaunchKernelGGL(moments_kernel, grid, dim3(kBlock), shm, st, (const double2 *)y, nshift, y_stride_l,
                     (const double2 *)c_dev, nmom, (double2 *)s, n, sl, sk);
}
void launch_moments_strided(const void *y, int nsrc, int nshift, const double *c_dev, int nmom, void *s,
                            int64_t n, int64_t sl, int64_t sk, hipStream_t st) {
  launch_moments_strided2(y, nsrc, nshift, nshift, c_dev, nmom, s, n, sl, sk, st);
}
void launch_moments(const void *y, int nsrc, int nshift, const double *c_dev, int nmom, void *s, int64_t n,
                    hipStream_t st) {
  launch_moments_strided(y, nsrc, nshift, c_dev, nmom, s, n, nmom, 1, st);
}

}  // namespace sscg
