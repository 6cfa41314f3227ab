// Tall-skinny FP64 complex products for the extraction stage (Sec. 2.1):
// Gram matrices S^H S and Q^H (A Q), basis changes S T, and column residuals.
// Matrices are "column-major over vectors": column a of an n x na matrix is the
// n-vector at A + a * lda (complex, interleaved). These run once per eigensolve;
// they are bandwidth-bound streaming passes over the n-length columns.
#include "sscg_internal.h"

namespace sscg {

// Both products tile their output in 64 x 64 blocks of 256 threads; a thread owns
// 4 x 4 outputs (rows/columns t + 16 i), and operands pass through LDS in steps of 16
// along the summed index, so every LDS read feeds four complex multiply-adds.
constexpr int kGT = 64;  // output tile edge
constexpr int kGK = 16;  // summed-index step staged in LDS

// partial[chunk][a][b] = sum over the chunk's rows of conj(A[row][a]) B[row][b].
// herm = 1 (a Hermitian product, na = nb): only the tiles on and above the diagonal
// (the caller mirrors the rest); the blocks enumerate them row by row.
// Held to 168 registers (three wavefronts per SIMD; the two registers it gives up are
// spilled outside the summation loop). One-dimensional grid of tiles x nchunk blocks,
// numbered so that the tiles of one row chunk run on one XCD (workgroups are dealt
// round-robin over the 8 XCDs, each with its own L2): the chunk's rows are then fetched
// from HBM once and re-read from that L2 by its other tiles.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gemm_cn_kernel(const double2 *__restrict__ A, int64_t lda, int na,
                                                      const double2 *__restrict__ B, int64_t ldb, int nb,
                                                      int64_t n, double2 *partial, int nchunk, int herm) {
  __shared__ double2 As[kGK][kGT + 1];
  __shared__ double2 Bs[kGK][kGT + 1];
  const int tiles_b = (nb + kGT - 1) / kGT;
  const int ntile = herm ? tiles_b * (tiles_b + 1) / 2 : ((na + kGT - 1) / kGT) * tiles_b;
  const int groups = nchunk / 8;  // chunks in groups of 8, one per XCD
  const int lin = blockIdx.x;
  int tile, chunk;
  if (lin < ntile * groups * 8) {
    const int xcd = lin & 7, s = lin >> 3;
    chunk = (s / ntile) * 8 + xcd;
    tile = s % ntile;
  } else {  // the chunks past the last group of 8, in plain order
    const int r = lin - ntile * groups * 8;
    chunk = groups * 8 + r / ntile;
    tile = r % ntile;
  }
  int ta = tile / tiles_b, tb = tile % tiles_b;
  if (herm) {
    ta = 0;
    tb = tile;
    while (tb >= tiles_b - ta) {  // row ta holds tiles ta .. tiles_b - 1
      tb -= tiles_b - ta;
      ++ta;
    }
    tb += ta;
  }
  const int a0 = ta * kGT, b0 = tb * kGT;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t rows_per = (n + nchunk - 1) / nchunk;
  const int64_t r_begin = (int64_t)chunk * rows_per;
  const int64_t r_end = min(n, r_begin + rows_per);
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0, 0);
  // loader: row (t & 15) of columns (t >> 4) + 16 q: 16 threads read 16 consecutive
  // rows; the next step's values are loaded into registers while this step computes
  const int lrow = t & 15, lcol = t >> 4;
  double2 pa[4], pb[4];
  auto fetch = [&](int64_t r0) {
    const int64_t row = r0 + lrow;
    const bool rv = row < r_end;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = lcol + 16 * q;
      pa[q] = (rv && a0 + col < na) ? A[(size_t)(a0 + col) * lda + row] : make_double2(0, 0);
      pb[q] = (rv && b0 + col < nb) ? B[(size_t)(b0 + col) * ldb + row] : make_double2(0, 0);
    }
  };
  if (r_begin < r_end) fetch(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[lrow][lcol + 16 * q] = pa[q];
      Bs[lrow][lcol + 16 * q] = pb[q];
    }
    __syncthreads();
    if (r0 + kGK < r_end) fetch(r0 + kGK);
#pragma unroll 4
    for (int k = 0; k < kGK; ++k) {
      double2 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfmac(acc[i][j], av[i], bv[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ty + 16 * i, b = b0 + tx + 16 * j;
      if (a < na && b < nb) partial[((size_t)chunk * na + a) * nb + b] = acc[i][j];
    }
}

// C[:, b] = sum_a A[:, a] T[a][b], T row-major (na x nb) in device memory. Block:
// 64 rows x 64 columns of C; thread t owns rows (t & 15) + 16 r and columns
// (t >> 4) + 16 c. upper = 1: T is upper triangular (T[a][b] = 0 for a > b), and the
// sum for a column tile stops at its last column (the skipped terms are zero).
__global__ __launch_bounds__(256) void gemm_nn_kernel(const double2 *__restrict__ A, int64_t lda, int na,
                                                      const double2 *__restrict__ T, int nb,
                                                      double2 *__restrict__ C, int64_t ldc, int64_t n,
                                                      int upper) {
  __shared__ double2 As[kGK][kGT + 1];  // [a][row]
  __shared__ double2 Ts[kGK][kGT + 1];  // [a][column]
  // one-dimensional grid, numbered so that the column tiles of one row tile run on one
  // XCD one after another (workgroups are dealt round-robin over the 8 XCDs): the row
  // tile's columns of A are fetched from HBM once and re-read from that XCD's L2
  const int64_t rtiles = (n + kGT - 1) / kGT;
  const int ctiles = (nb + kGT - 1) / kGT;
  const int64_t groups = rtiles / 8, lin = blockIdx.x;
  int64_t rt;
  int ctl;
  if (lin < groups * 8 * ctiles) {
    const int64_t s = lin >> 3;
    rt = (s / ctiles) * 8 + (lin & 7);
    ctl = (int)(s % ctiles);
  } else {  // the row tiles past the last group of 8, in plain order
    const int64_t r = lin - groups * 8 * ctiles;
    rt = groups * 8 + r / ctiles;
    ctl = (int)(r % ctiles);
  }
  const int64_t i0 = rt * kGT;
  const int b0 = ctl * kGT;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0, 0);
  // loader: 64 consecutive rows (or columns) of 4 values of the summed index; the
  // next step's values are loaded into registers while this step computes
  const int lx = t & 63, lk = t >> 6;
  double2 pa[4], pt[4];
  auto fetch = [&](int ka) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = ka + lk + 4 * q;
      const int64_t row = i0 + lx;
      pa[q] = (a < na && row < n) ? A[(size_t)a * lda + row] : make_double2(0, 0);
      pt[q] = (a < na && b0 + lx < nb) ? T[(size_t)a * nb + b0 + lx] : make_double2(0, 0);
    }
  };
  const int kend = upper ? min(na, b0 + kGT) : na;
  fetch(0);
  for (int ka = 0; ka < kend; ka += kGK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[lk + 4 * q][lx] = pa[q];
      Ts[lk + 4 * q][lx] = pt[q];
    }
    __syncthreads();
    if (ka + kGK < kend) fetch(ka + kGK);
#pragma unroll 4
    for (int k = 0; k < kGK; ++k) {
      double2 av[4], tv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[k][tx + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) tv[c] = Ts[k][ty + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cfma(acc[r][c], av[r], tv[c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int b = b0 + ty + 16 * c;
    if (b >= nb) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = i0 + tx + 16 * r;
      if (row < n) C[(size_t)b * ldc + row] = acc[r][c];
    }
  }
}

__global__ void colscale_kernel(double2 *A, int64_t lda, const double *scale, int64_t n) {
  const int a = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    double2 v = A[(size_t)a * lda + i];
    v.x *= scale[a];
    v.y *= scale[a];
    A[(size_t)a * lda + i] = v;
  }
}

// partial[c][chunk] = ||AX[:,c] - lam_c X[:,c]||^2 over the chunk (and [ncol + c] = ||X[:,c]||^2)
__global__ __launch_bounds__(256) void resid_cols_kernel(const double2 *AX, const double2 *X, int64_t ld,
                                                         int ncol, const double *lam, int64_t n,
                                                         double *partial, int nchunk) {
  __shared__ double red[8];
  const int c = blockIdx.y, chunk = blockIdx.x;
  const double l = lam[c];
  double acc = 0.0, nx = 0.0;
  for (int64_t i = (int64_t)chunk * 256 + threadIdx.x; i < n; i += (int64_t)nchunk * 256) {
    const double2 x = X[(size_t)c * ld + i], ax = AX[(size_t)c * ld + i];
    const double rx = ax.x - l * x.x, ry = ax.y - l * x.y;
    acc += rx * rx + ry * ry;
    nx += x.x * x.x + x.y * x.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc += __shfl_xor(acc, off, 64);
    nx += __shfl_xor(nx, off, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { red[w] = acc; red[4 + w] = nx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[(size_t)c * nchunk + chunk] = red[0] + red[1] + red[2] + red[3];
    partial[(size_t)(ncol + c) * nchunk + chunk] = red[4] + red[5] + red[6] + red[7];
  }
}

// out[o] = sum_k partial[k][o] for o < nout (partials laid out [nchunk][nout]); doubles.
// Block of 256 threads per 64 outputs: wavefront w sums the chunks k = w mod 4 (four
// independent load streams per output), then the four sums are added in a fixed order.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *partial, int nchunk, int nout,
                                                              double *out) {
  __shared__ double red[4][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int o = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (o < nout)
    for (int k = w; k < nchunk; k += 4) s += partial[(size_t)k * nout + o];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && o < nout) out[o] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

void launch_gemm_cn(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nb, int64_t n,
                    double *partial, int nchunk, int herm, hipStream_t st) {
  const int tiles = gemm_cn_tiles(na, nb, herm);
  hipLaunchKernelGGL(gemm_cn_kernel, dim3(tiles * nchunk), dim3(256), 0, st, (const double2 *)A, lda, na,
                     (const double2 *)B, ldb, nb, n, (double2 *)partial, nchunk, herm);
}
void launch_gemm_nn(const void *A, int64_t lda, int na, const double *T, int nb, void *C, int64_t ldc,
                    int64_t n, int upper, hipStream_t st) {
  if (n <= 0 || na <= 0 || nb <= 0) return;
  const dim3 grid((unsigned)(((n + kGT - 1) / kGT) * ((nb + kGT - 1) / kGT)));
  hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(256), 0, st, (const double2 *)A, lda, na, (const double2 *)T, nb,
                     (double2 *)C, ldc, n, upper);
}
int gemm_cn_tiles(int na, int nb, int herm) {
  const int ta = (na + kGT - 1) / kGT, tb = (nb + kGT - 1) / kGT;
  return herm ? ta * (ta + 1) / 2 : ta * tb;
}
void launch_colscale(void *A, int64_t lda, int na, const double *scale, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)((n + 255) / 256), na), dim3(256), 0, st, (double2 *)A,
                     lda, scale, n);
}
void launch_resid_cols(const void *AX, const void *X, int64_t ld, int ncol, const double *lam, int64_t n,
                       double *partial, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(resid_cols_kernel, dim3(nchunk, ncol), dim3(256), 0, st, (const double2 *)AX,
                     (const double2 *)X, ld, ncol, lam, n, partial, nchunk);
}
void launch_reduce_partials(const double *partial, int nchunk, int nout, double *out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((nout + 63) / 64), dim3(256), 0, st, partial, nchunk, nout,
                     out);
}

}  // namespace sscg
