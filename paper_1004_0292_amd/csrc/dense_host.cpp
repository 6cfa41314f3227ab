// Host FP64 eigen-decomposition of small Hermitian matrices, used for the
// projected matrices of the Rayleigh-Ritz and Hankel extraction (Sec. 2.1);
// sizes are at most M*L (a few hundred).
//
// Method: Householder reduction to a real symmetric tridiagonal matrix followed
// by the implicit QL iteration with shifts (the tql2 scheme of Bowdler, Martin,
// Reinsch and Wilkinson, 1968), then back-transformation of the eigenvectors.
//   1. For k = 0 .. n-3 a reflector H_k = I - beta v v^H maps column k below the
//      diagonal onto alpha e_1 and is applied to the trailing block as a
//      Hermitian rank-2 update; A = Q T Q^H with Q = H_0 ... H_{n-3}.
//   2. The complex sub-diagonal of T is made real by a diagonal unitary D:
//      T = D T_r D^H with T_r real symmetric tridiagonal.
//   3. QL with implicit shifts diagonalises T_r = Z diag(lambda) Z^T.
//   4. Eigenvectors of A are the columns of Q D Z.
//
// Matrices are column-major, complex as interleaved doubles: element (i, j) is
// A[2 (i + n j)] + i A[2 (i + n j) + 1].
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

namespace sscg {

namespace {
struct cpx {
  double re, im;
};
inline cpx cadd(cpx a, cpx b) { return {a.re + b.re, a.im + b.im}; }
inline cpx csub(cpx a, cpx b) { return {a.re - b.re, a.im - b.im}; }
inline cpx cmul(cpx a, cpx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cpx cmulc(cpx a, cpx b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a) b
inline cpx cscal(cpx a, double s) { return {a.re * s, a.im * s}; }
inline double cabs(cpx a) { return std::hypot(a.re, a.im); }
}  // namespace

void herm_eig(int n, const double *Ain, double *evals, double *evecs) {
  if (n <= 0) return;
  std::vector<cpx> A((size_t)n * n);
  auto a = [&](int i, int j) -> cpx & { return A[(size_t)i + (size_t)n * j]; };
  // Hermitian part of the input
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) a(i, j) = {Ain[2 * ((size_t)i + (size_t)n * j)], Ain[2 * ((size_t)i + (size_t)n * j) + 1]};
  for (int j = 0; j < n; ++j) {
    a(j, j).im = 0.0;
    for (int i = j + 1; i < n; ++i) {
      const cpx lo = a(i, j), up = a(j, i);
      const cpx h = {0.5 * (lo.re + up.re), 0.5 * (lo.im - up.im)};
      a(i, j) = h;
      a(j, i) = {h.re, -h.im};
    }
  }
  // 1. Householder tridiagonalisation
  std::vector<cpx> V((size_t)n * n, {0.0, 0.0});  // reflector k stored in column k, rows k+1..n-1
  std::vector<double> beta(n, 0.0);
  std::vector<cpx> p(n), w(n);
  std::vector<double> d(n, 0.0), e(n, 0.0);
  std::vector<cpx> sub(n, {0.0, 0.0});  // complex sub-diagonal T[k+1][k]
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = A[k+1.., k]
    double sig2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const cpx x = a(k + 1 + i, k);
      sig2 += x.re * x.re + x.im * x.im;
    }
    const double sig = std::sqrt(sig2);
    const cpx x0 = a(k + 1, k);
    const double ax0 = cabs(x0);
    if (sig == 0.0) {
      sub[k] = {0.0, 0.0};
      continue;
    }
    const cpx ph = ax0 > 0 ? cpx{x0.re / ax0, x0.im / ax0} : cpx{1.0, 0.0};
    const cpx alpha = cscal(ph, -sig);
    cpx *v = &V[(size_t)n * k + k + 1];
    for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
    v[0] = csub(v[0], alpha);
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i].re * v[i].re + v[i].im * v[i].im;
    if (vv == 0.0) {
      sub[k] = x0;
      continue;
    }
    const double b = 2.0 / vv;
    beta[k] = b;
    // p = b A22 v, A22 = A[k+1.., k+1..]
    for (int i = 0; i < m; ++i) p[i] = {0.0, 0.0};
    for (int j = 0; j < m; ++j) {
      const cpx vj = v[j];
      const cpx *col = &A[(size_t)(k + 1) + (size_t)n * (k + 1 + j)];
      for (int i = 0; i < m; ++i) p[i] = cadd(p[i], cmul(col[i], vj));
    }
    cpx vp = {0.0, 0.0};
    for (int i = 0; i < m; ++i) {
      p[i] = cscal(p[i], b);
      vp = cadd(vp, cmulc(v[i], p[i]));
    }
    // w = p - (b/2) (v^H p) v ; A22 <- A22 - v w^H - w v^H
    const double K = 0.5 * b * vp.re;
    for (int i = 0; i < m; ++i) w[i] = csub(p[i], cscal(v[i], K));
    for (int j = 0; j < m; ++j) {
      const cpx wj = w[j], vj = v[j];
      cpx *col = &A[(size_t)(k + 1) + (size_t)n * (k + 1 + j)];
      for (int i = 0; i < m; ++i) {
        // v_i conj(w_j) + w_i conj(v_j)
        const cpx t1 = {v[i].re * wj.re + v[i].im * wj.im, v[i].im * wj.re - v[i].re * wj.im};
        const cpx t2 = {w[i].re * vj.re + w[i].im * vj.im, w[i].im * vj.re - w[i].re * vj.im};
        col[i] = csub(col[i], cadd(t1, t2));
      }
    }
    sub[k] = alpha;
  }
  for (int k = 0; k < n; ++k) d[k] = a(k, k).re;
  if (n >= 2) sub[n - 2] = a(n - 1, n - 2);
  // 2. real sub-diagonal through phases delta_{k+1} = delta_k e_k / |e_k|
  std::vector<cpx> delta(n, {1.0, 0.0});
  for (int k = 0; k + 1 < n; ++k) {
    const double ae = cabs(sub[k]);
    e[k] = ae;
    delta[k + 1] = ae > 0 ? cmul(delta[k], cpx{sub[k].re / ae, sub[k].im / ae}) : delta[k];
  }
  e[n - 1] = 0.0;
  // 3. implicit QL on (d, e); Z accumulates the rotations (column-major n x n)
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i + (size_t)n * i] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) break;  // does not happen for Hermitian input; guards the loop
      // shift from the leading 2x2 block of the unreduced part
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i], bb = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * bb;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - bb;
        double *zi = &Z[(size_t)n * i], *zi1 = &Z[(size_t)n * (i + 1)];
        for (int k = 0; k < n; ++k) {
          const double t = zi1[k];
          zi1[k] = s * zi[k] + c * t;
          zi[k] = c * zi[k] - s * t;
        }
      }
      if (deflated) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int k = 0; k < n; ++k) evals[k] = d[order[k]];
  if (!evecs) return;
  // 4. eigenvectors: X = Q D Z (columns in ascending eigenvalue order)
  std::vector<cpx> X((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    const double *zc = &Z[(size_t)n * order[k]];
    cpx *xc = &X[(size_t)n * k];
    for (int i = 0; i < n; ++i) xc[i] = cscal(delta[i], zc[i]);
  }
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const int m = n - k - 1;
    const cpx *v = &V[(size_t)n * k + k + 1];
    for (int c = 0; c < n; ++c) {
      cpx *xc = &X[(size_t)n * c + k + 1];
      cpx s = {0.0, 0.0};
      for (int i = 0; i < m; ++i) s = cadd(s, cmulc(v[i], xc[i]));
      s = cscal(s, beta[k]);
      for (int i = 0; i < m; ++i) xc[i] = csub(xc[i], cmul(v[i], s));
    }
  }
  for (size_t t = 0; t < (size_t)n * n; ++t) {
    evecs[2 * t] = X[t].re;
    evecs[2 * t + 1] = X[t].im;
  }
}

}  // namespace sscg
