// Tall-skinny FP64 complex products for the extraction stage (Sec. 2.1):
// Gram matrices S^H S and Q^H (A Q), basis changes S T, and column residuals.
// Matrices are "column-major over vectors": column a of an n x na matrix is the
// n-vector at A + a * lda (complex, interleaved). These run once per eigensolve;
// they are bandwidth-bound streaming passes over the n-length columns.
#include "sscg_internal.h"

namespace sscg {

constexpr int kT = 16;  // output tile edge for the Gram kernel

// partial[chunk][a][b] = sum over the chunk's rows of conj(A[row][a]) B[row][b]
__global__ __launch_bounds__(256) void gemm_cn_kernel(const double2 *__restrict__ A, int64_t lda, int na,
                                                      const double2 *__restrict__ B, int64_t ldb, int nb,
                                                      int64_t n, double2 *partial, int nchunk) {
  __shared__ double2 As[kT][kT + 1];
  __shared__ double2 Bs[kT][kT + 1];
  const int tiles_b = (nb + kT - 1) / kT;
  const int tile = blockIdx.x, chunk = blockIdx.y;
  const int a0 = (tile / tiles_b) * kT, b0 = (tile % tiles_b) * kT;
  const int tx = threadIdx.x & (kT - 1), ty = threadIdx.x / kT;
  const int64_t rows_per = (n + nchunk - 1) / nchunk;
  const int64_t r_begin = (int64_t)chunk * rows_per;
  const int64_t r_end = min(n, r_begin + rows_per);
  double2 acc = make_double2(0, 0);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kT) {
    // load: thread (ty, tx) fetches row r0 + tx of column a0 + ty (and b0 + ty)
    const int64_t row = r0 + tx;
    const bool rv = row < r_end;
    As[ty][tx] = (rv && a0 + ty < na) ? A[(size_t)(a0 + ty) * lda + row] : make_double2(0, 0);
    Bs[ty][tx] = (rv && b0 + ty < nb) ? B[(size_t)(b0 + ty) * ldb + row] : make_double2(0, 0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kT; ++k) cfmac(acc, As[ty][k], Bs[tx][k]);
    __syncthreads();
  }
  const int a = a0 + ty, b = b0 + tx;
  if (a < na && b < nb) partial[((size_t)chunk * na + a) * nb + b] = acc;
}

// C[:, b] = sum_a A[:, a] T[a][b], T row-major (na x nb) in device memory.
constexpr int kNB = 16;
__global__ __launch_bounds__(256) void gemm_nn_kernel(const double2 *__restrict__ A, int64_t lda, int na,
                                                      const double2 *__restrict__ T, int nb,
                                                      double2 *__restrict__ C, int64_t ldc, int64_t n) {
  extern __shared__ double2 Ts[];  // [na][kNB]
  const int b0 = blockIdx.y * kNB;
  const int nbl = min(kNB, nb - b0);
  for (int t = threadIdx.x; t < na * kNB; t += 256) {
    const int a = t / kNB, bb = t - a * kNB;
    Ts[t] = bb < nbl ? T[(size_t)a * nb + b0 + bb] : make_double2(0, 0);
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double2 acc[kNB];
#pragma unroll
  for (int bb = 0; bb < kNB; ++bb) acc[bb] = make_double2(0, 0);
  for (int a = 0; a < na; ++a) {
    const double2 av = A[(size_t)a * lda + i];
#pragma unroll
    for (int bb = 0; bb < kNB; ++bb) cfma(acc[bb], av, Ts[a * kNB + bb]);
  }
#pragma unroll
  for (int bb = 0; bb < kNB; ++bb)
    if (bb < nbl) C[(size_t)(b0 + bb) * ldc + i] = acc[bb];
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

// out[o] = sum_k partial[k][o] for o < nout (partials laid out [nchunk][nout]); doubles
__global__ void reduce_partials_kernel(const double *partial, int nchunk, int nout, double *out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += partial[(size_t)k * nout + o];
  out[o] = s;
}

void launch_gemm_cn(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nb, int64_t n,
                    double *partial, int nchunk, hipStream_t st) {
  const int tiles = ((na + kT - 1) / kT) * ((nb + kT - 1) / kT);
  hipLaunchKernelGGL(gemm_cn_kernel, dim3(tiles, nchunk), dim3(256), 0, st, (const double2 *)A, lda, na,
                     (const double2 *)B, ldb, nb, n, (double2 *)partial, nchunk);
}
void launch_gemm_nn(const void *A, int64_t lda, int na, const double *T, int nb, void *C, int64_t ldc,
                    int64_t n, hipStream_t st) {
  const dim3 grid((unsigned)((n + 255) / 256), (nb + kNB - 1) / kNB);
  const size_t shm = (size_t)na * kNB * sizeof(double2);
  hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(256), shm, st, (const double2 *)A, lda, na,
                     (const double2 *)T, nb, (double2 *)C, ldc, n);
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
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((nout + 255) / 256), dim3(256), 0, st, partial, nchunk,
                     nout, out);
}

}  // namespace sscg
