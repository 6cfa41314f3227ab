// Host FP64 eigen-decomposition of small Hermitian matrices, used for the
// projected matrices of the Rayleigh-Ritz and Hankel extraction (Sec. 2.1);
// sizes are at most M*L (a few hundred).
//
// Method: Householder reduction to a real symmetric tridiagonal matrix, the
// implicit symmetric QR iteration with Wilkinson shifts on it, then
// back-transformation of the eigenvectors.
//   1. For k = 0 .. n-3 a reflector H_k = I - beta v v^H maps column k below the
//      diagonal onto alpha e_1 and is applied to the trailing block as a
//      Hermitian rank-2 update; A = Q T Q^H with Q = H_0 ... H_{n-3}.
//   2. The complex sub-diagonal of T is made real by a diagonal unitary D:
//      T = D T_r D^H with T_r real symmetric tridiagonal.
//   3. Implicit QR steps diagonalise T_r = Z diag(lambda) Z^T. Each step works on
//      the trailing unreduced block [lo, hi] (off-diagonal entries below
//      eps (|a_k| + |a_{k+1}|) count as zero): the shift mu is the eigenvalue of
//      the block's last 2x2 corner nearer to a_hi; a rotation in the plane
//      (lo, lo+1) taken from the first column (a_lo - mu, b_lo) of T - mu I
//      starts the step, and rotations in the planes (k, k+1) then move the
//      off-tridiagonal entry it creates down the block until it leaves at the
//      bottom. T stays symmetric tridiagonal, the step equals one shifted QR
//      step on the block, and b_{hi-1} falls off quickly (cubically near the end).
//   4. Eigenvectors of A are the columns of Q D Z.
//
// Matrices are column-major, complex as interleaved doubles: element (i, j) is
// A[2 (i + n j)] + i A[2 (i + n j) + 1]. Internally the real and imaginary parts
// are held in separate arrays, and the eigenvectors are back-transformed in
// row-major order, so that every inner loop runs over contiguous memory without a
// reduction (the loops vectorise).
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "host_math.h"

namespace sscg {

namespace {
// sqrt(a^2 + b^2), without the cost of std::hypot where the squares cannot over- or
// underflow
inline double hyp(double a, double b) {
  const double m = std::fmax(std::fabs(a), std::fabs(b));
  if (m > 1e-150 && m < 1e150) return std::sqrt(a * a + b * b);
  return std::hypot(a, b);
}
}  // namespace

// Built twice, for AVX2 with FMA and for plain x86-64; the loader picks the first at
// run time where the processor has it (one plain build when SSCG_NO_TARGET_CLONES is
// defined, as in the sanitizer build of the host code).
#ifdef SSCG_NO_TARGET_CLONES
#define SSCG_HOST_CLONES
#else
#define SSCG_HOST_CLONES __attribute__((target_clones("arch=x86-64-v3", "default")))
#endif
SSCG_HOST_CLONES bool herm_eig(int n, const double *Ain, double *evals, double *evecs) {
  if (n <= 0) return true;
  const size_t nn = (size_t)n * n;
  std::vector<double> Ar(nn), Ai(nn);  // column-major, split real / imaginary parts
  // Hermitian part of the input
  auto id = [n](int i, int j) { return (size_t)i + (size_t)n * j; };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      Ar[id(i, j)] = Ain[2 * id(i, j)];
      Ai[id(i, j)] = Ain[2 * id(i, j) + 1];
    }
  for (int j = 0; j < n; ++j) {
    Ai[id(j, j)] = 0.0;
    for (int i = j + 1; i < n; ++i) {
      const double hr = 0.5 * (Ar[id(i, j)] + Ar[id(j, i)]), hi = 0.5 * (Ai[id(i, j)] - Ai[id(j, i)]);
      Ar[id(i, j)] = hr; Ai[id(i, j)] = hi;
      Ar[id(j, i)] = hr; Ai[id(j, i)] = -hi;
    }
  }
  // 1. Householder tridiagonalisation: reflector k in column k of V, rows k+1..n-1;
  // (sr, si) the complex sub-diagonal T[k+1][k]
  std::vector<double> Vr(nn, 0.0), Vi(nn, 0.0), beta(n, 0.0);
  std::vector<double> pr(n), pi(n), wr(n), wi(n), d(n, 0.0), e(n, 0.0), sr(n, 0.0), si(n, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const double *xr = &Ar[id(k + 1, k)], *xi = &Ai[id(k + 1, k)];
    double sig2 = 0.0;
    for (int i = 0; i < m; ++i) sig2 += xr[i] * xr[i] + xi[i] * xi[i];
    const double sig = std::sqrt(sig2);
    const double x0r = xr[0], x0i = xi[0];
    const double ax0 = hyp(x0r, x0i);
    if (sig == 0.0) { sr[k] = si[k] = 0.0; continue; }
    const double phr = ax0 > 0 ? x0r / ax0 : 1.0, phi = ax0 > 0 ? x0i / ax0 : 0.0;
    const double alr = -sig * phr, ali = -sig * phi;
    double *vr = &Vr[id(k + 1, k)], *vi = &Vi[id(k + 1, k)];
    for (int i = 0; i < m; ++i) { vr[i] = xr[i]; vi[i] = xi[i]; }
    vr[0] -= alr; vi[0] -= ali;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += vr[i] * vr[i] + vi[i] * vi[i];
    if (vv == 0.0) { sr[k] = x0r; si[k] = x0i; continue; }
    const double b = 2.0 / vv;
    beta[k] = b;
    // p = b A22 v with A22 = A[k+1.., k+1..]
    for (int i = 0; i < m; ++i) pr[i] = pi[i] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double vjr = vr[j], vji = vi[j];
      const double *cr = &Ar[id(k + 1, k + 1 + j)], *ci = &Ai[id(k + 1, k + 1 + j)];
      for (int i = 0; i < m; ++i) {
        pr[i] += cr[i] * vjr - ci[i] * vji;
        pi[i] += cr[i] * vji + ci[i] * vjr;
      }
    }
    double vpr = 0.0;
    for (int i = 0; i < m; ++i) {
      pr[i] *= b; pi[i] *= b;
      vpr += vr[i] * pr[i] + vi[i] * pi[i];
    }
    // w = p - (b/2) (v^H p) v ; A22 <- A22 - v w^H - w v^H
    const double K = 0.5 * b * vpr;
    for (int i = 0; i < m; ++i) { wr[i] = pr[i] - K * vr[i]; wi[i] = pi[i] - K * vi[i]; }
    for (int j = 0; j < m; ++j) {
      const double wjr = wr[j], wji = wi[j], vjr = vr[j], vji = vi[j];
      double *cr = &Ar[id(k + 1, k + 1 + j)], *ci = &Ai[id(k + 1, k + 1 + j)];
      for (int i = 0; i < m; ++i) {
        cr[i] -= (vr[i] * wjr + vi[i] * wji) + (wr[i] * vjr + wi[i] * vji);
        ci[i] -= (vi[i] * wjr - vr[i] * wji) + (wi[i] * vjr - wr[i] * vji);
      }
    }
    sr[k] = alr; si[k] = ali;
  }
  for (int k = 0; k < n; ++k) d[k] = Ar[id(k, k)];
  if (n >= 2) { sr[n - 2] = Ar[id(n - 1, n - 2)]; si[n - 2] = Ai[id(n - 1, n - 2)]; }
  // 2. real sub-diagonal through the phases delta_{k+1} = delta_k e_k / |e_k|
  std::vector<double> dr(n, 1.0), di(n, 0.0);
  for (int k = 0; k + 1 < n; ++k) {
    const double ae = hyp(sr[k], si[k]);
    e[k] = ae;
    if (ae > 0) {
      const double ur = sr[k] / ae, ui = si[k] / ae;
      dr[k + 1] = dr[k] * ur - di[k] * ui;
      di[k + 1] = dr[k] * ui + di[k] * ur;
    } else { dr[k + 1] = dr[k]; di[k + 1] = di[k]; }
  }
  e[n - 1] = 0.0;
  // 3. implicit symmetric QR on (d, e): d the diagonal, e[k] the entry (k, k+1);
  // Z accumulates the rotations (column-major n x n)
  std::vector<double> Z(nn, 0.0);
  for (int i = 0; i < n; ++i) Z[id(i, i)] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  auto negligible = [&](int k) { return std::fabs(e[k]) <= eps * (std::fabs(d[k]) + std::fabs(d[k + 1])); };
  // rotation G = [[c, s], [-s, c]] in the plane (k, k+1): T <- G T G^T, Z <- Z G^T
  auto rotate_z = [&](int k, double c, double s) {
    double *zk = &Z[id(0, k)], *zk1 = &Z[id(0, k + 1)];
    for (int q = 0; q < n; ++q) {
      const double u = zk[q], v = zk1[q];
      zk[q] = c * u + s * v;
      zk1[q] = c * v - s * u;
    }
  };
  bool converged = true;
  long steps = 0;
  const long max_steps = 30L * n + 30;
  int hi = n - 1;
  while (hi > 0) {
    if (negligible(hi - 1)) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(lo - 1)) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    if (++steps > max_steps) {
      converged = false;
      break;
    }
    // Wilkinson shift: eigenvalue of [[d_{hi-1}, e_{hi-1}], [e_{hi-1}, d_hi]] nearer d_hi
    const double half = 0.5 * (d[hi - 1] - d[hi]), bb = e[hi - 1];
    const double den = half + (half >= 0.0 ? hyp(half, bb) : -hyp(half, bb));
    const double mu = d[hi] - bb * (bb / den);
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hyp(x, z);
      const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? z / r : 0.0;
      if (k > lo) e[k - 1] = r;  // the entry (k-1, k+1) is rotated away
      const double ak = d[k], ak1 = d[k + 1], bk = e[k];
      const double cc = c * c, ss = s * s, cs = c * s;
      d[k] = cc * ak + 2.0 * cs * bk + ss * ak1;
      d[k + 1] = ss * ak - 2.0 * cs * bk + cc * ak1;
      e[k] = cs * (ak1 - ak) + (cc - ss) * bk;
      if (k + 1 < hi) {  // the rotation creates the entry (k, k+2) = s e_{k+1}
        z = s * e[k + 1];
        e[k + 1] *= c;
        x = e[k];
      }
      rotate_z(k, c, s);
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int k = 0; k < n; ++k) evals[k] = d[order[k]];
  if (!evecs) return converged;
  // 4. eigenvectors X = Q D Z (columns in ascending eigenvalue order), held
  // row-major (X[i][c] at i n + c) so the reflector sums run over contiguous columns
  std::vector<double> Xr(nn), Xi(nn), tr(n), ti(n);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < n; ++c) {
      const double z = Z[id(i, order[c])];
      Xr[(size_t)i * n + c] = dr[i] * z;
      Xi[(size_t)i * n + c] = di[i] * z;
    }
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const int m = n - k - 1;
    const double *vr = &Vr[id(k + 1, k)], *vi = &Vi[id(k + 1, k)];
    for (int c = 0; c < n; ++c) tr[c] = ti[c] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double a = vr[i], bq = vi[i];
      const double *xr = &Xr[(size_t)(k + 1 + i) * n], *xi = &Xi[(size_t)(k + 1 + i) * n];
      for (int c = 0; c < n; ++c) {  // t += conj(v_i) x_i
        tr[c] += a * xr[c] + bq * xi[c];
        ti[c] += a * xi[c] - bq * xr[c];
      }
    }
    const double b = beta[k];
    for (int c = 0; c < n; ++c) { tr[c] *= b; ti[c] *= b; }
    for (int i = 0; i < m; ++i) {
      const double a = vr[i], bq = vi[i];
      double *xr = &Xr[(size_t)(k + 1 + i) * n], *xi = &Xi[(size_t)(k + 1 + i) * n];
      for (int c = 0; c < n; ++c) {  // x_i -= v_i t
        xr[c] -= a * tr[c] - bq * ti[c];
        xi[c] -= a * ti[c] + bq * tr[c];
      }
    }
  }
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      evecs[2 * id(i, c)] = Xr[(size_t)i * n + c];
      evecs[2 * id(i, c) + 1] = Xi[(size_t)i * n + c];
    }
  return converged;
}
}  // namespace sscg
