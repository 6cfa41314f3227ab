// Wilson dslash for the Hermitian fermion matrix A = gamma5 (I - kappa D) (Sec. 4).
//
// One thread per lattice site, NR sources per thread (the links of a site are
// loaded once and applied to NR spinors). Every hop uses the rank-2 spin
// projector (1 -+ gamma_mu): two colour vectors are formed from the neighbour
// spinor, multiplied by U_mu(x) (forward) or U_mu(x-mu)^H (backward), and the
// four spin components are rebuilt from them. Chiral basis:
//   (1 - g1) psi = [h0, h1,  i h1,  i h0],  h0 = p0 - i p3,  h1 = p1 - i p2
//   (1 + g1) psi = [h0, h1, -i h1, -i h0],  h0 = p0 + i p3,  h1 = p1 + i p2
//   (1 - g2) psi = [h0, h1, -h1,  h0],      h0 = p0 + p3,    h1 = p1 - p2
//   (1 + g2) psi = [h0, h1,  h1, -h0],      h0 = p0 - p3,    h1 = p1 + p2
//   (1 - g3) psi = [h0, h1,  i h0, -i h1],  h0 = p0 - i p2,  h1 = p1 + i p3
//   (1 + g3) psi = [h0, h1, -i h0,  i h1],  h0 = p0 + i p2,  h1 = p1 - i p3
//   (1 - g4) psi = [h0, h1, -h0, -h1],      h0 = p0 - p2,    h1 = p1 - p3
//   (1 + g4) psi = [h0, h1,  h0,  h1],      h0 = p0 + p2,    h1 = p1 + p3
// Epilogue: out = A psi = gamma5 (psi - kappa D psi) (mode 0), or the CG seed
// matrix out = sigma psi - A psi (mode 1), with partial sums of Re <psi, out> per
// 64-site wavefront written for the CG step length when requested.
//
// Memory: the spinor planes and link planes are site-contiguous, so each of the
// 8 neighbour gathers of a wavefront is a run of 64 consecutive complex numbers
// (shifted by the hop); neighbour reuse is left to L2. Blocks are renumbered so
// that consecutive site tiles land on the same XCD (the hardware deals blocks
// round-robin over the 8 XCDs, each with its own L2).
#include <algorithm>

#include "sscg_internal.h"

namespace sscg {

// Non-temporal (streaming) store of one complex number: the output spinor is not
// re-read by this launch, so it need not take L2 space from the neighbours' spinors.
template <typename C>
__device__ __forceinline__ void st_stream(C *p, C v) {
  typedef decltype(v.x) E;
  typedef E ev2 __attribute__((ext_vector_type(2)));
  ev2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<ev2 *>(p));
}

// A solve-loop launch carries one extra block (the last) that commits the staged
// state of the previous iteration of every job; the other blocks read only the done
// flags, so at worst they compute a finished source once more, whose result is not
// used.
__device__ __forceinline__ void commit_batch(const DslashBatch &B) {
  for (int k = 0; k < B.njobs; ++k)
    if (B.job[k].shift) commit_states(B.job[k].seed, B.job[k].shift, B.job[k].nsrc, B.job[k].nshift);
}

__device__ __forceinline__ int xcd_remap_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7;
  const int x = b & 7, local = b >> 3;
  return x * q + (x < rem ? x : rem) + local;
}

template <typename T, int LR>
__device__ __forceinline__ void load_link(const V2<T> *__restrict__ g, int V, int mu, int s,
                                          V2<T> (&u)[9]) {
  const V2<T> *base = g + (size_t)mu * (LR / 2) * V + s;
#pragma unroll
  for (int e = 0; e < LR / 2; ++e) u[e] = base[(size_t)e * V];
  if constexpr (LR == 12) {
    // third row of an SU(3) matrix: conj(row0 x row1)
    V2<T> c0 = cmul(u[1], u[5]) - cmul(u[2], u[4]);
    V2<T> c1 = cmul(u[2], u[3]) - cmul(u[0], u[5]);
    V2<T> c2 = cmul(u[0], u[4]) - cmul(u[1], u[3]);
    u[6] = cmk<V2<T>>(c0.x, -c0.y);
    u[7] = cmk<V2<T>>(c1.x, -c1.y);
    u[8] = cmk<V2<T>>(c2.x, -c2.y);
  }
}

// h0, h1 of the projector (1 + sgn gamma_mu), sgn = -1 forward, +1 backward.
template <int MU, int SGN, typename C>
__device__ __forceinline__ void project(const C (&p)[12], C (&h0)[3], C (&h1)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if constexpr (MU == 0) {
      if constexpr (SGN < 0) { h0[c] = p0 + cmi(p3); h1[c] = p1 + cmi(p2); }
      else                   { h0[c] = p0 + ci(p3);  h1[c] = p1 + ci(p2); }
    } else if constexpr (MU == 1) {
      if constexpr (SGN < 0) { h0[c] = p0 + p3; h1[c] = p1 - p2; }
      else                   { h0[c] = p0 - p3; h1[c] = p1 + p2; }
    } else if constexpr (MU == 2) {
      if constexpr (SGN < 0) { h0[c] = p0 + cmi(p2); h1[c] = p1 + ci(p3); }
      else                   { h0[c] = p0 + ci(p2);  h1[c] = p1 + cmi(p3); }
    } else {
      if constexpr (SGN < 0) { h0[c] = p0 - p2; h1[c] = p1 - p3; }
      else                   { h0[c] = p0 + p2; h1[c] = p1 + p3; }
    }
  }
}

// acc (12 components, 3 spin + colour) += (1 + sgn gamma_mu) rebuilt from g0, g1.
template <int MU, int SGN, typename C>
__device__ __forceinline__ void reconstruct(C (&acc)[12], const C (&g0)[3], const C (&g1)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] = acc[c] + g0[c];
    acc[3 + c] = acc[3 + c] + g1[c];
    if constexpr (MU == 0) {
      if constexpr (SGN < 0) { acc[6 + c] = acc[6 + c] + ci(g1[c]);  acc[9 + c] = acc[9 + c] + ci(g0[c]); }
      else                   { acc[6 + c] = acc[6 + c] + cmi(g1[c]); acc[9 + c] = acc[9 + c] + cmi(g0[c]); }
    } else if constexpr (MU == 1) {
      if constexpr (SGN < 0) { acc[6 + c] = acc[6 + c] - g1[c]; acc[9 + c] = acc[9 + c] + g0[c]; }
      else                   { acc[6 + c] = acc[6 + c] + g1[c]; acc[9 + c] = acc[9 + c] - g0[c]; }
    } else if constexpr (MU == 2) {
      if constexpr (SGN < 0) { acc[6 + c] = acc[6 + c] + ci(g0[c]);  acc[9 + c] = acc[9 + c] + cmi(g1[c]); }
      else                   { acc[6 + c] = acc[6 + c] + cmi(g0[c]); acc[9 + c] = acc[9 + c] + ci(g1[c]); }
    } else {
      if constexpr (SGN < 0) { acc[6 + c] = acc[6 + c] - g0[c]; acc[9 + c] = acc[9 + c] - g1[c]; }
      else                   { acc[6 + c] = acc[6 + c] + g0[c]; acc[9 + c] = acc[9 + c] + g1[c]; }
    }
  }
}

template <typename C>
__device__ __forceinline__ void su3_mul(const C (&u)[9], const C (&h)[3], C (&g)[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    C a = cmul(u[3 * i], h[0]);
    cfma(a, u[3 * i + 1], h[1]);
    cfma(a, u[3 * i + 2], h[2]);
    g[i] = a;
  }
}
template <typename C>
__device__ __forceinline__ void su3_mul_adj(const C (&u)[9], const C (&h)[3], C (&g)[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    C a = cmulc(u[i], h[0]);
    cfmac(a, u[3 + i], h[1]);
    cfmac(a, u[6 + i], h[2]);
    g[i] = a;
  }
}

template <typename T, int NR, int LR, int MU>
__device__ __forceinline__ void hop(const V2<T> *__restrict__ in, const V2<T> *__restrict__ gauge,
                                    int V, int s, int sf, int sb, int nvalid,
                                    V2<T> (&acc)[NR][12]) {
  using C = V2<T>;
  C u[9];
  // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
  load_link<T, LR>(gauge, V, MU, s, u);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nvalid) {
      const C *src = in + (size_t)r * 12 * V + sf;
      C p[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c] = src[(size_t)c * V];
      C h0[3], h1[3], g0[3], g1[3];
      project<MU, -1>(p, h0, h1);
      su3_mul(u, h0, g0);
      su3_mul(u, h1, g1);
      reconstruct<MU, -1>(acc[r], g0, g1);
    }
  }
  // backward: (1 + gamma_mu) U_mu(x - mu)^H psi(x - mu)
  load_link<T, LR>(gauge, V, MU, sb, u);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nvalid) {
      const C *src = in + (size_t)r * 12 * V + sb;
      C p[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c] = src[(size_t)c * V];
      C h0[3], h1[3], g0[3], g1[3];
      project<MU, 1>(p, h0, h1);
      su3_mul_adj(u, h0, g0);
      su3_mul_adj(u, h1, g1);
      reconstruct<MU, 1>(acc[r], g0, g1);
    }
  }
}

template <typename T, int NR, int LR, int BS>
__global__ __launch_bounds__(BS) void dslash_kernel(DslashBatch B, int xcd_remap) {
  using C = V2<T>;
  int b = blockIdx.x;
  if (B.commit && b == B.total_blocks) {
    commit_batch(B);
    return;
  }
  if (xcd_remap) b = xcd_remap_block(b, B.total_blocks);
  int begins[kMaxJobs];
#pragma unroll
  for (int k = 0; k < kMaxJobs; ++k) begins[k] = B.job[k].block_begin;
  const int ji = find_job(begins, B.njobs, b);
  const DslashJob &J = B.job[ji];
  const int lb = b - J.block_begin;
  // site-major order (J.order = 1): the source groups of one site tile are adjacent
  // blocks, so after the XCD renumbering one XCD serves all sources of a lattice
  // region and fetches its links once; group-major (0): one source at a time
  const int groups = (J.nsrc + NR - 1) / NR;
  int group, sblk;
  if (J.order == 1) {
    sblk = lb / groups;
    group = lb - sblk * groups;
  } else {
    group = lb / J.nblk_site;
    sblk = lb - group * J.nblk_site;
  }
  const int l0 = group * NR;
  const int nvalid = min(NR, J.nsrc - l0);
  if (J.seed) {
    bool all_done = true;
    for (int r = 0; r < nvalid; ++r) all_done &= (J.seed[l0 + r].done != 0);
    if (all_done) return;
  }
  const int V = J.V;
  const int s = sblk * BS + threadIdx.x;
  const bool valid = s < V;
  const V2<T> *in = reinterpret_cast<const V2<T> *>(J.in) + (size_t)l0 * 12 * V;
  V2<T> *out = reinterpret_cast<V2<T> *>(J.out) + (size_t)l0 * 12 * V;
  const V2<T> *gauge = reinterpret_cast<const V2<T> *>(J.gauge);

  double dot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) dot[r] = 0.0;

  if (valid) {
    const int Lx = J.dims[0], Ly = J.dims[1], Lz = J.dims[2], Lt = J.dims[3];
    const int x = s % Lx, t1 = s / Lx, y = t1 % Ly, t2 = t1 / Ly, z = t2 % Lz, t = t2 / Lz;
    const int sx = 1, sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
    const int fx = s + (x == Lx - 1 ? (1 - Lx) * sx : sx), bx = s + (x == 0 ? (Lx - 1) * sx : -sx);
    const int fy = s + (y == Ly - 1 ? (1 - Ly) * sy : sy), by = s + (y == 0 ? (Ly - 1) * sy : -sy);
    const int fz = s + (z == Lz - 1 ? (1 - Lz) * sz : sz), bz = s + (z == 0 ? (Lz - 1) * sz : -sz);
    const int ft = s + (t == Lt - 1 ? (1 - Lt) * st : st), bt = s + (t == 0 ? (Lt - 1) * st : -st);

    C acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[r][c] = cmk<C>(0, 0);

    hop<T, NR, LR, 0>(in, gauge, V, s, fx, bx, nvalid, acc);
    hop<T, NR, LR, 1>(in, gauge, V, s, fy, by, nvalid, acc);
    hop<T, NR, LR, 2>(in, gauge, V, s, fz, bz, nvalid, acc);
    hop<T, NR, LR, 3>(in, gauge, V, s, ft, bt, nvalid, acc);

    const T kap = (T)J.kappa;
    const T sig = (T)J.sigma;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nvalid) {
        const C *src = in + (size_t)r * 12 * V + s;
        C *dst = out + (size_t)r * 12 * V + s;
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const C p = src[(size_t)c * V];
          const C a = acc[r][c];
          C o;
          if (J.mode == 1) {
            // sigma psi - gamma5 (psi - kappa D psi)
            if (c < 6) { o.x = (sig - (T)1) * p.x + kap * a.x; o.y = (sig - (T)1) * p.y + kap * a.y; }
            else       { o.x = (sig + (T)1) * p.x - kap * a.x; o.y = (sig + (T)1) * p.y - kap * a.y; }
          } else {
            if (c < 6) { o.x = p.x - kap * a.x; o.y = p.y - kap * a.y; }
            else       { o.x = kap * a.x - p.x; o.y = kap * a.y - p.y; }
          }
          st_stream(dst + (size_t)c * V, o);
          d += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
        }
        dot[r] = d;
      }
    }
  }
  if (J.partial) {
    // one partial per 64-site wavefront, at the wave's global index: the layout and
    // the summation order do not depend on the block size or sources per thread
    const int wave = s >> 6;
    const int npart = (V + 63) >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double d = dot[r];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
      if ((threadIdx.x & 63) == 0 && r < nvalid && wave < npart) J.partial[(size_t)(l0 + r) * npart + wave] = d;
    }
  }
}

// Direction-split variant for small lattices (latency-bound: too few sites to fill
// the chip with one thread per site). A block owns 64 sites and NR sources; each of
// its 4 wavefronts takes one direction mu (forward and backward hop), the four
// 12-component results are added in LDS in a fixed order, and wavefront w then
// finishes output components 3w .. 3w+2. One partial of Re <psi, out> per 64 sites,
// as in the other kernels.
template <typename T, int NR, int LR>
__global__ __launch_bounds__(256) void dslash_split_kernel(DslashBatch B, int xcd_remap) {
  using C = V2<T>;
  __shared__ C red[4][NR * 12][64];
  __shared__ double dsum[4][NR];
  int b = blockIdx.x;
  if (B.commit && b == B.total_blocks) {
    commit_batch(B);
    return;
  }
  if (xcd_remap) b = xcd_remap_block(b, B.total_blocks);
  int begins[kMaxJobs];
#pragma unroll
  for (int k = 0; k < kMaxJobs; ++k) begins[k] = B.job[k].block_begin;
  const int ji = find_job(begins, B.njobs, b);
  const DslashJob &J = B.job[ji];
  const int lb = b - J.block_begin;
  const int groups = (J.nsrc + NR - 1) / NR;
  const int sblk = lb / groups, group = lb - sblk * groups;
  const int l0 = group * NR;
  const int nvalid = min(NR, J.nsrc - l0);
  if (J.seed) {
    bool all_done = true;
    for (int r = 0; r < nvalid; ++r) all_done &= (J.seed[l0 + r].done != 0);
    if (all_done) return;  // uniform over the block, before any barrier
  }
  const int V = J.V;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int s = sblk * 64 + lane;
  const bool valid = s < V;
  const V2<T> *in = reinterpret_cast<const V2<T> *>(J.in) + (size_t)l0 * 12 * V;
  V2<T> *out = reinterpret_cast<V2<T> *>(J.out) + (size_t)l0 * 12 * V;
  const V2<T> *gauge = reinterpret_cast<const V2<T> *>(J.gauge);
  C acc[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[r][c] = cmk<C>(0, 0);
  if (valid) {
    const int Lx = J.dims[0], Ly = J.dims[1], Lz = J.dims[2], Lt = J.dims[3];
    const int x = s % Lx, t1 = s / Lx, y = t1 % Ly, t2 = t1 / Ly, z = t2 % Lz, t = t2 / Lz;
    if (wv == 0) {
      hop<T, NR, LR, 0>(in, gauge, V, s, s + (x == Lx - 1 ? 1 - Lx : 1), s + (x == 0 ? Lx - 1 : -1), nvalid, acc);
    } else if (wv == 1) {
      const int sy = Lx;
      hop<T, NR, LR, 1>(in, gauge, V, s, s + (y == Ly - 1 ? (1 - Ly) * sy : sy), s + (y == 0 ? (Ly - 1) * sy : -sy),
                        nvalid, acc);
    } else if (wv == 2) {
      const int sz = Lx * Ly;
      hop<T, NR, LR, 2>(in, gauge, V, s, s + (z == Lz - 1 ? (1 - Lz) * sz : sz), s + (z == 0 ? (Lz - 1) * sz : -sz),
                        nvalid, acc);
    } else {
      const int st = Lx * Ly * Lz;
      hop<T, NR, LR, 3>(in, gauge, V, s, s + (t == Lt - 1 ? (1 - Lt) * st : st), s + (t == 0 ? (Lt - 1) * st : -st),
                        nvalid, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) red[wv][r * 12 + c][lane] = acc[r][c];
  __syncthreads();
  const T kap = (T)J.kappa;
  const T sig = (T)J.sigma;
  double dot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    dot[r] = 0.0;
    if (r < nvalid && valid) {
      const C *src = in + (size_t)r * 12 * V + s;
      C *dst = out + (size_t)r * 12 * V + s;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const int c = 3 * wv + cc;
        C a = red[0][r * 12 + c][lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) a = a + red[w][r * 12 + c][lane];
        const C p = src[(size_t)c * V];
        C o;
        if (J.mode == 1) {
          if (c < 6) { o.x = (sig - (T)1) * p.x + kap * a.x; o.y = (sig - (T)1) * p.y + kap * a.y; }
          else       { o.x = (sig + (T)1) * p.x - kap * a.x; o.y = (sig + (T)1) * p.y - kap * a.y; }
        } else {
          if (c < 6) { o.x = p.x - kap * a.x; o.y = p.y - kap * a.y; }
          else       { o.x = kap * a.x - p.x; o.y = kap * a.y - p.y; }
        }
        st_stream(dst + (size_t)c * V, o);
        dot[r] += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
      }
    }
  }
  if (J.partial) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double d = dot[r];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
      if (lane == 0) dsum[wv][r] = d;
    }
    __syncthreads();
    const int npart = (V + 63) >> 6;
    if (threadIdx.x < NR && (int)threadIdx.x < nvalid) {
      const int r = threadIdx.x;
      J.partial[(size_t)(l0 + r) * npart + sblk] = ((dsum[0][r] + dsum[1][r]) + dsum[2][r]) + dsum[3][r];
    }
  }
}

// One spatial direction of the tile kernel: a neighbour inside the block's tile is
// read from the block's LDS copy of the current slice (local index lf / lb >= 0),
// one outside it from memory (site sf / sb).
template <typename T, int NR, int LR, int MU>
__device__ __forceinline__ void hop_tile(const V2<T> *__restrict__ in, const V2<T> *__restrict__ gauge,
                                         const V2<T> *lds, int V, int BS, int s, int sf, int sb, int lf, int lb,
                                         int nvalid, V2<T> (&acc)[NR][12]) {
  using C = V2<T>;
  C u[9];
  load_link<T, LR>(gauge, V, MU, s, u);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nvalid) {
      C p[12];
      if (lf >= 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = lds[(r * 12 + c) * BS + lf];
      } else {
        const C *src = in + (size_t)r * 12 * V + sf;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = src[(size_t)c * V];
      }
      C h0[3], h1[3], g0[3], g1[3];
      project<MU, -1>(p, h0, h1);
      su3_mul(u, h0, g0);
      su3_mul(u, h1, g1);
      reconstruct<MU, -1>(acc[r], g0, g1);
    }
  }
  load_link<T, LR>(gauge, V, MU, sb, u);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nvalid) {
      C p[12];
      if (lb >= 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = lds[(r * 12 + c) * BS + lb];
      } else {
        const C *src = in + (size_t)r * 12 * V + sb;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = src[(size_t)c * V];
      }
      C h0[3], h1[3], g0[3], g1[3];
      project<MU, 1>(p, h0, h1);
      su3_mul_adj(u, h0, g0);
      su3_mul_adj(u, h1, g1);
      reconstruct<MU, 1>(acc[r], g0, g1);
    }
  }
}

// local index of a neighbour inside the tile, or -1; the tile spans the whole
// lattice in that direction when T == L (then the neighbour wraps inside it)
__device__ __forceinline__ int tile_nb(int tid, int l, int T, int L, int stride, bool fwd) {
  if (T == L) return fwd ? tid + (l == T - 1 ? (1 - T) * stride : stride) : tid + (l == 0 ? (T - 1) * stride : -stride);
  if (fwd) return l < T - 1 ? tid + stride : -1;
  return l > 0 ? tid - stride : -1;
}

// Tile-marching variant (J.ct > 0). A block owns a spatial tile of whole x-rows,
// Lx x ty x tz sites with one thread per site, and walks it through ct
// consecutive time slices:
//  * t-hops from registers: the spinor of slice t+1 loaded for the forward hop is
//    the centre spinor of the next step, and the backward hop into slice t+1,
//    U_t(x, t)^H (1 + gamma_4) psi(x, t), is formed while slice t is current, with
//    the t-link already loaded for the forward hop of slice t;
//  * x, y, z hops from LDS: each step the block stores its centre spinors of the
//    current slice in LDS, and neighbours inside the tile are read from there;
//    only the faces of the tile (1/ty and 1/tz of the sites per direction) read
//    their neighbours from memory.
// So every spinor is read from memory about once per block, plus the two slices
// bounding the t-range and the tile faces. Needs ty | Ly, tz | Lz and Lx ty tz a
// multiple of 64 (at most 1024); dynamic LDS of nr * 12 * Lx ty tz complex numbers.
// Partials of Re <psi, out>: one per 64-site wavefront, indexed by (slice, tile,
// wavefront), V / 64 of them as in the site-parallel kernel.
// FP32 tiles with one source per thread fit three wavefronts per SIMD in 168
// registers; the bound keeps the compiler there (a register more would cost a
// wavefront per SIMD on 256-thread tiles).
template <typename T, int NR, int MAXBS>
constexpr int tile_min_blocks() { return (sizeof(T) == 4 && NR == 1 && MAXBS == 256) ? 3 : 1; }

template <typename T, int NR, int LR, int MAXBS>
__global__ __launch_bounds__(MAXBS, (tile_min_blocks<T, NR, MAXBS>())) void dslash_tile_kernel(DslashBatch B,
                                                                                              int xcd_remap) {
  using C = V2<T>;
  extern __shared__ __align__(16) unsigned char dslash_lds[];
  C *lds = reinterpret_cast<C *>(dslash_lds);
  int b = blockIdx.x;
  if (B.commit && b == B.total_blocks) {
    commit_batch(B);
    return;
  }
  if (xcd_remap) b = xcd_remap_block(b, B.total_blocks);
  int begins[kMaxJobs];
#pragma unroll
  for (int k = 0; k < kMaxJobs; ++k) begins[k] = B.job[k].block_begin;
  const int ji = find_job(begins, B.njobs, b);
  const DslashJob &J = B.job[ji];
  const int lb = b - J.block_begin;
  const int Lx = J.dims[0], Ly = J.dims[1], Lz = J.dims[2], Lt = J.dims[3];
  const int Ty = J.ty, Tz = J.tz;
  const int BS = Lx * Ty * Tz;
  const int nty = Ly / Ty, ntile = nty * (Lz / Tz);
  const int nrange = (Lt + J.ct - 1) / J.ct;
  const int groups = (J.nsrc + NR - 1) / NR;
  // block order (J.order): 1 = source groups innermost, then tiles, then t-ranges
  // (one XCD serves all sources of a region, links fetched once); 0 = source
  // groups outermost; 2 = source groups outermost, t-ranges innermost
  int group, range, tile;
  if (J.order == 1) {
    const int sg = lb / groups;
    group = lb - sg * groups;
    range = sg / ntile;
    tile = sg - range * ntile;
  } else {
    const int per = ntile * nrange;
    group = lb / per;
    const int sg = lb - group * per;
    if (J.order == 0) {
      range = sg / ntile;
      tile = sg - range * ntile;
    } else {
      tile = sg / nrange;
      range = sg - tile * nrange;
    }
  }
  const int t0 = range * J.ct, t1 = min(t0 + J.ct, Lt);
  const int l0 = group * NR;
  const int nvalid = min(NR, J.nsrc - l0);
  if (J.seed) {
    bool all_done = true;
    for (int r = 0; r < nvalid; ++r) all_done &= (J.seed[l0 + r].done != 0);
    if (all_done) return;  // uniform over the block, before any barrier
  }
  const int V = J.V;
  const int Vs = Lx * Ly * Lz;
  const int tid = threadIdx.x;
  const int lx = tid % Lx, q = tid / Lx, ly = q % Ty, lz = q / Ty;
  const int x = lx, y = (tile % nty) * Ty + ly, z = (tile / nty) * Tz + lz;
  const int sp = x + Lx * (y + Ly * z);
  const int sxy = Lx * Ly;
  const int fx = sp + (x == Lx - 1 ? 1 - Lx : 1), bx = sp + (x == 0 ? Lx - 1 : -1);
  const int fy = sp + (y == Ly - 1 ? (1 - Ly) * Lx : Lx), by = sp + (y == 0 ? (Ly - 1) * Lx : -Lx);
  const int fz = sp + (z == Lz - 1 ? (1 - Lz) * sxy : sxy), bz = sp + (z == 0 ? (Lz - 1) * sxy : -sxy);
  const int lfx = tile_nb(tid, lx, Lx, Lx, 1, true), lbx = tile_nb(tid, lx, Lx, Lx, 1, false);
  const int lfy = tile_nb(tid, ly, Ty, Ly, Lx, true), lby = tile_nb(tid, ly, Ty, Ly, Lx, false);
  const int lfz = tile_nb(tid, lz, Tz, Lz, Lx * Ty, true), lbz = tile_nb(tid, lz, Tz, Lz, Lx * Ty, false);
  const V2<T> *in = reinterpret_cast<const V2<T> *>(J.in) + (size_t)l0 * 12 * V;
  V2<T> *out = reinterpret_cast<V2<T> *>(J.out) + (size_t)l0 * 12 * V;
  const V2<T> *gauge = reinterpret_cast<const V2<T> *>(J.gauge);
  const int npart = V >> 6;
  const int wpt = BS >> 6;

  C bw0[NR][3], bw1[NR][3];
  C u[9];
  {
    // backward t-hop into slice t0; the centre spinors of slice t0 go to LDS
    const int sprev = sp + Vs * (t0 == 0 ? Lt - 1 : t0 - 1);
    load_link<T, LR>(gauge, V, 3, sprev, u);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nvalid) {
        const C *src = in + (size_t)r * 12 * V + sprev;
        C p[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = src[(size_t)c * V];
        C h0[3], h1[3];
        project<3, 1>(p, h0, h1);
        su3_mul_adj(u, h0, bw0[r]);
        su3_mul_adj(u, h1, bw1[r]);
        const C *cs = in + (size_t)r * 12 * V + sp + Vs * t0;
#pragma unroll
        for (int c = 0; c < 12; ++c) lds[(r * 12 + c) * BS + tid] = cs[(size_t)c * V];
      }
    }
  }
  const T kap = (T)J.kappa;
  const T sig = (T)J.sigma;
  for (int t = t0; t < t1; ++t) {
    const int ofs = Vs * t;
    const int s = sp + ofs;
    const int sn = sp + Vs * (t == Lt - 1 ? 0 : t + 1);
    // spinors of slice t+1 (forward t-hop now, the centre of the next step)
    C nxt[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nvalid) {
        const C *src = in + (size_t)r * 12 * V + sn;
#pragma unroll
        for (int c = 0; c < 12; ++c) nxt[r][c] = src[(size_t)c * V];
      }
    }
    __syncthreads();  // slice t of the tile is in LDS
    C acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[r][c] = cmk<C>(0, 0);
    hop_tile<T, NR, LR, 0>(in, gauge, lds, V, BS, s, fx + ofs, bx + ofs, lfx, lbx, nvalid, acc);
    hop_tile<T, NR, LR, 1>(in, gauge, lds, V, BS, s, fy + ofs, by + ofs, lfy, lby, nvalid, acc);
    hop_tile<T, NR, LR, 2>(in, gauge, lds, V, BS, s, fz + ofs, bz + ofs, lfz, lbz, nvalid, acc);
    load_link<T, LR>(gauge, V, 3, s, u);
    double dot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dot[r] = 0.0;
      if (r < nvalid) {
        C h0[3], h1[3], g0[3], g1[3];
        project<3, -1>(nxt[r], h0, h1);
        su3_mul(u, h0, g0);
        su3_mul(u, h1, g1);
        reconstruct<3, -1>(acc[r], g0, g1);
        reconstruct<3, 1>(acc[r], bw0[r], bw1[r]);
        C cur[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) cur[c] = lds[(r * 12 + c) * BS + tid];
        if (t + 1 < t1) {
          project<3, 1>(cur, h0, h1);
          su3_mul_adj(u, h0, bw0[r]);
          su3_mul_adj(u, h1, bw1[r]);
        }
        C *dst = out + (size_t)r * 12 * V + s;
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const C p = cur[c];
          const C a = acc[r][c];
          C o;
          if (J.mode == 1) {
            if (c < 6) { o.x = (sig - (T)1) * p.x + kap * a.x; o.y = (sig - (T)1) * p.y + kap * a.y; }
            else       { o.x = (sig + (T)1) * p.x - kap * a.x; o.y = (sig + (T)1) * p.y - kap * a.y; }
          } else {
            if (c < 6) { o.x = p.x - kap * a.x; o.y = p.y - kap * a.y; }
            else       { o.x = kap * a.x - p.x; o.y = kap * a.y - p.y; }
          }
          st_stream(dst + (size_t)c * V, o);
          d += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
        }
        dot[r] = d;
      }
    }
    if (J.partial) {
      const int wave = (t * ntile + tile) * wpt + (tid >> 6);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double d = dot[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
        if ((tid & 63) == 0 && r < nvalid) J.partial[(size_t)(l0 + r) * npart + wave] = d;
      }
    }
    __syncthreads();  // every read of slice t is done: slice t+1 replaces it
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nvalid)
#pragma unroll
        for (int c = 0; c < 12; ++c) lds[(r * 12 + c) * BS + tid] = nxt[r][c];
  }
}

template <typename T, int NR, int LR, int MAXBS>
static void launch_tile(const DslashBatch &b, int bs, size_t shm, int xcd, hipStream_t st) {
  // dynamic LDS above the default needs the kernel attribute; it is raised once per
  // instantiation to the most this instantiation can ask for (NR sources of MAXBS
  // sites), so every tile size it launches is covered (the device limit is checked
  // by the caller's tile choice)
  static bool raised = false;
  constexpr size_t kMaxShm = (size_t)NR * 12 * MAXBS * sizeof(V2<T>);
  if (kMaxShm > 65536 && !raised) {
    int dev = 0, lim = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lim = 65536;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&dslash_tile_kernel<T, NR, LR, MAXBS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::min(kMaxShm, (size_t)lim));
    raised = true;
  }
  hipLaunchKernelGGL((dslash_tile_kernel<T, NR, LR, MAXBS>), dim3(b.total_blocks + b.commit), dim3(bs), shm, st, b, xcd);
}

template <typename T, int NR, int LR>
static void launch_m(const DslashBatch &b, int xcd, hipStream_t st) {
  const DslashJob &j = b.job[0];
  const int bs = j.dims[0] * j.ty * j.tz;
  const size_t shm = (size_t)NR * 12 * bs * sizeof(V2<T>);
  if (bs <= 256) launch_tile<T, NR, LR, 256>(b, bs, shm, xcd, st);
  else if (bs <= 512) launch_tile<T, NR, LR, 512>(b, bs, shm, xcd, st);
  else if (bs <= 768) launch_tile<T, NR, LR, 768>(b, bs, shm, xcd, st);
  else launch_tile<T, NR, LR, 1024>(b, bs, shm, xcd, st);
}

template <typename T, int NR, int LR>
static void launch_t(const DslashBatch &b, int bs, int xcd, hipStream_t st) {
  if (bs == 64)
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 64>), dim3(b.total_blocks + b.commit), dim3(64), 0, st, b, xcd);
  else if (bs == 128)
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 128>), dim3(b.total_blocks + b.commit), dim3(128), 0, st, b, xcd);
  else
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 256>), dim3(b.total_blocks + b.commit), dim3(256), 0, st, b, xcd);
}

template <typename T, int LR>
static void launch_nr(const DslashBatch &b, int nr, int bs, int xcd, int ct, hipStream_t st) {
  if (ct < 0) {
    if (nr == 1)
      hipLaunchKernelGGL((dslash_split_kernel<T, 1, LR>), dim3(b.total_blocks + b.commit), dim3(256), 0, st, b, xcd);
    else
      hipLaunchKernelGGL((dslash_split_kernel<T, 2, LR>), dim3(b.total_blocks + b.commit), dim3(256), 0, st, b, xcd);
    return;
  }
  if (ct > 0) {
    if (nr == 1) launch_m<T, 1, LR>(b, xcd, st);
    else if (nr == 2) launch_m<T, 2, LR>(b, xcd, st);
    else launch_m<T, 4, LR>(b, xcd, st);
    return;
  }
  if (nr == 1) launch_t<T, 1, LR>(b, bs, xcd, st);
  else if (nr == 2) launch_t<T, 2, LR>(b, bs, xcd, st);
  else launch_t<T, 4, LR>(b, bs, xcd, st);
}

void launch_dslash(const DslashBatch &b, int prec, int nr, int lr, int bs, int xcd, int ct, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  if (prec == 0) launch_nr<double, 18>(b, nr, bs, xcd, ct, st);
  else if (lr == 18) launch_nr<float, 18>(b, nr, bs, xcd, ct, st);
  else launch_nr<float, 12>(b, nr, bs, xcd, ct, st);
}

}  // namespace sscg
