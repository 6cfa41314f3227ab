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
#include "sscg_internal.h"

namespace sscg {

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
  if (xcd_remap) b = xcd_remap_block(b, gridDim.x);
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
  if (J.order) {
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
  const int ii = sblk * BS + threadIdx.x;  // position in the traversal order
  const bool valid = ii < V;
  // Traversal order: with px > 0 the lattice is walked in x-pieces of width px
  // (order: piece, t, z, y, x within the piece), which shortens the distance between
  // a site and its t- and z-neighbours in the order the blocks run; otherwise
  // lexicographic. The data layout itself is lexicographic either way.
  int s = ii;
  if (J.px > 0 && valid) {
    const int px = J.px, Ly = J.dims[1], Lz = J.dims[2], Lt = J.dims[3];
    const int xl = ii % px;
    int r2 = ii / px;
    const int yy = r2 % Ly;
    r2 /= Ly;
    const int zz = r2 % Lz;
    r2 /= Lz;
    const int tt = r2 % Lt;
    const int pc = r2 / Lt;
    s = pc * px + xl + J.dims[0] * (yy + Ly * (zz + Lz * tt));
  }
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
          dst[(size_t)c * V] = o;
          d += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
        }
        dot[r] = d;
      }
    }
  }
  if (J.partial) {
    // one partial per 64-site wavefront, at the wave's global index: the layout and
    // the summation order do not depend on the block size or sources per thread
    const int wave = ii >> 6;
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

template <typename T, int NR, int LR>
static void launch_t(const DslashBatch &b, int bs, int xcd, hipStream_t st) {
  if (bs == 64)
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 64>), dim3(b.total_blocks), dim3(64), 0, st, b, xcd);
  else if (bs == 128)
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 128>), dim3(b.total_blocks), dim3(128), 0, st, b, xcd);
  else
    hipLaunchKernelGGL((dslash_kernel<T, NR, LR, 256>), dim3(b.total_blocks), dim3(256), 0, st, b, xcd);
}

template <typename T, int LR>
static void launch_nr(const DslashBatch &b, int nr, int bs, int xcd, hipStream_t st) {
  if (nr == 1) launch_t<T, 1, LR>(b, bs, xcd, st);
  else if (nr == 2) launch_t<T, 2, LR>(b, bs, xcd, st);
  else launch_t<T, 4, LR>(b, bs, xcd, st);
}

void launch_dslash(const DslashBatch &b, int prec, int nr, int lr, int bs, int xcd, hipStream_t st) {
  if (b.total_blocks <= 0) return;
  if (prec == 0) launch_nr<double, 18>(b, nr, bs, xcd, st);
  else if (lr == 18) launch_nr<float, 18>(b, nr, bs, xcd, st);
  else launch_nr<float, 12>(b, nr, bs, xcd, st);
}

}  // namespace sscg
