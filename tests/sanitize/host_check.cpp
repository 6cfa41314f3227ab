// Host-code check run under AddressSanitizer and UndefinedBehaviorSanitizer (built
// with g++ by tests/test_sanitize_host.py): the dense Hermitian eigensolver, the
// quadrature of the lines and the circle, and the Cholesky factor of the
// Rayleigh-Ritz orthogonalisation, on sizes and inputs the library meets. Prints one
// line per check and exits non-zero on the first failure.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "host_math.h"

using sscg::cd;

static int fails = 0;
static void check(bool ok, const char *what, double val) {
  printf("%s %s %.3e\n", ok ? "ok  " : "FAIL", what, val);
  if (!ok) ++fails;
}

// column-major Hermitian matrix with a given spectrum: Q diag(lam) Q^H, Q from a
// Gram-Schmidt of random columns
static std::vector<cd> hermitian(int n, const std::vector<double> &lam, std::mt19937_64 &g) {
  std::normal_distribution<double> nd;
  std::vector<cd> Q((size_t)n * n);
  for (auto &q : Q) q = cd(nd(g), nd(g));
  for (int c = 0; c < n; ++c) {
    for (int pass = 0; pass < 2; ++pass)
      for (int d = 0; d < c; ++d) {
        cd dot = 0;
        for (int i = 0; i < n; ++i) dot += std::conj(Q[i + (size_t)n * d]) * Q[i + (size_t)n * c];
        for (int i = 0; i < n; ++i) Q[i + (size_t)n * c] -= dot * Q[i + (size_t)n * d];
      }
    double nr = 0;
    for (int i = 0; i < n; ++i) nr += std::norm(Q[i + (size_t)n * c]);
    for (int i = 0; i < n; ++i) Q[i + (size_t)n * c] /= std::sqrt(nr);
  }
  std::vector<cd> A((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int k = 0; k < n; ++k) s += Q[i + (size_t)n * k] * lam[k] * std::conj(Q[j + (size_t)n * k]);
      A[i + (size_t)n * j] = s;
    }
  return A;
}

int main() {
  std::mt19937_64 g(7);
  for (int n : {1, 2, 3, 7, 40, 130, 256}) {
    std::vector<double> lam(n);
    for (int k = 0; k < n; ++k) lam[k] = (k % 2 ? -1.0 : 1.0) * std::pow(10.0, -10.0 * k / std::max(1, n - 1));
    std::vector<cd> A = hermitian(n, lam, g);
    std::vector<double> ev(n), vec(2 * (size_t)n * n);
    const bool conv = sscg::herm_eig(n, reinterpret_cast<const double *>(A.data()), ev.data(), vec.data());
    const cd *V = reinterpret_cast<const cd *>(vec.data());
    double res = 0, orth = 0;
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) {
        cd s = 0;
        for (int j = 0; j < n; ++j) s += A[i + (size_t)n * j] * V[j + (size_t)n * k];
        res = std::max(res, std::abs(s - ev[k] * V[i + (size_t)n * k]));
      }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        cd s = 0;
        for (int i = 0; i < n; ++i) s += std::conj(V[i + (size_t)n * a]) * V[i + (size_t)n * b];
        orth = std::max(orth, std::abs(s - (a == b ? 1.0 : 0.0)));
      }
    char what[64];
    snprintf(what, sizeof what, "herm_eig n=%d residual", n);
    check(conv && res < 1e-12, what, res);
    snprintf(what, sizeof what, "herm_eig n=%d orthogonality", n);
    check(orth < 1e-12, what, orth);
  }
  for (int N : {4, 16, 32, 64}) {
    std::vector<cd> z, zeta, w;
    sscg::quad_lines_host(N, 0.1, 0.2, 0.3, z, zeta, w);
    // sum_j w_j zeta_j^(k-1) = delta_k0 for k < N, in relative terms
    double err = 0;
    for (int k = 0; k < N; ++k) {
      cd s = 0;
      double mag = 0;
      for (int j = 0; j < N; ++j) {
        const cd t = w[j] * std::pow(zeta[j], k - 1);
        s += t;
        mag = std::max(mag, std::abs(t));
      }
      err = std::max(err, std::abs(s - (k == 0 ? 1.0 : 0.0)) / std::max(mag, 1.0));
    }
    char what[64];
    snprintf(what, sizeof what, "quad_lines N=%d weight system", N);
    check(err < 1e-9, what, err);
    sscg::quad_circle_host(N, 0.0, 1.0, z, zeta, w);
    double werr = 0;
    for (int j = 0; j < N; ++j) werr = std::max(werr, std::abs(w[j] - zeta[j] / (double)N));
    snprintf(what, sizeof what, "quad_circle N=%d weights", N);
    check(werr < 1e-15, what, werr);
  }
  for (int n : {1, 5, 64, 192}) {
    std::vector<double> lam(n);
    for (int k = 0; k < n; ++k) lam[k] = 1.0 + k;
    std::vector<cd> Acm = hermitian(n, lam, g), G((size_t)n * n), Rinv;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) G[(size_t)i * n + j] = Acm[i + (size_t)n * j];   // row-major
    const bool ok = sscg::chol_inverse_upper(n, G, Rinv);
    // Rinv^H G Rinv = I
    double err = 0;
    std::vector<cd> T((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cd s = 0;
        for (int k = 0; k < n; ++k) s += G[(size_t)i * n + k] * Rinv[(size_t)k * n + j];
        T[(size_t)i * n + j] = s;
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cd s = 0;
        for (int k = 0; k < n; ++k) s += std::conj(Rinv[(size_t)k * n + i]) * T[(size_t)k * n + j];
        err = std::max(err, std::abs(s - (i == j ? 1.0 : 0.0)));
      }
    char what[64];
    snprintf(what, sizeof what, "cholesky n=%d Rinv^H G Rinv = I", n);
    check(ok && err < 1e-12, what, err);
  }
  printf("%d failures\n", fails);
  return fails ? 1 : 0;
}
