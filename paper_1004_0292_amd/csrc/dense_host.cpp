// Host FP64 eigen-decomposition of small Hermitian matrices (cyclic Jacobi).
// Used for the projected matrices of the Rayleigh-Ritz and Hankel extraction
// (Sec. 2.1): sizes are at most M*L (a few hundred), so an O(n^3)-per-sweep
// Jacobi method is fast enough and is accurate to rounding in every eigenvalue.
//
// Matrices are column-major, complex as interleaved doubles: element (i, j) is
// A[2 (i + n j)] + i A[2 (i + n j) + 1].
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace sscg {

using cd = std::complex<double>;

void herm_eig(int n, const double *Ain, double *evals, double *evecs) {
  std::vector<cd> A(static_cast<size_t>(n) * n), Vm(static_cast<size_t>(n) * n, cd(0.0, 0.0));
  auto a = [&](int i, int j) -> cd & { return A[i + static_cast<size_t>(n) * j]; };
  auto v = [&](int i, int j) -> cd & { return Vm[i + static_cast<size_t>(n) * j]; };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) a(i, j) = cd(Ain[2 * (i + n * j)], Ain[2 * (i + n * j) + 1]);
  // Hermitian part (the input is Hermitian up to rounding)
  for (int j = 0; j < n; ++j) {
    a(j, j) = cd(a(j, j).real(), 0.0);
    for (int i = j + 1; i < n; ++i) {
      const cd h = 0.5 * (a(i, j) + std::conj(a(j, i)));
      a(i, j) = h;
      a(j, i) = std::conj(h);
    }
  }
  for (int i = 0; i < n; ++i) v(i, i) = 1.0;
  double fro = 0.0;
  for (auto &x : A) fro += std::norm(x);
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        if (i != j) off += std::norm(a(i, j));
    if (std::sqrt(off) <= 1e-17 * fro || fro == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const cd b = a(p, q);
        const double ab = std::abs(b);
        if (ab == 0.0) continue;
        const double app = a(p, p).real(), aqq = a(q, q).real();
        // phase that makes the (p, q) entry real and positive
        const cd ph = b / ab;  // e^{i phi}
        const double tau = (aqq - app) / (2.0 * ab);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // G = diag(1, conj(ph)) [[c, s], [-s, c]]
        const cd gpp = c, gpq = s, gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
        for (int i = 0; i < n; ++i) {  // columns: A <- A G
          const cd xp = a(i, p), xq = a(i, q);
          a(i, p) = xp * gpp + xq * gqp;
          a(i, q) = xp * gpq + xq * gqq;
        }
        for (int j = 0; j < n; ++j) {  // rows: A <- G^H A
          const cd xp = a(p, j), xq = a(q, j);
          a(p, j) = std::conj(gpp) * xp + std::conj(gqp) * xq;
          a(q, j) = std::conj(gpq) * xp + std::conj(gqq) * xq;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        a(p, p) = cd(a(p, p).real(), 0.0);
        a(q, q) = cd(a(q, q).real(), 0.0);
        for (int i = 0; i < n; ++i) {
          const cd xp = v(i, p), xq = v(i, q);
          v(i, p) = xp * gpp + xq * gqp;
          v(i, q) = xp * gpq + xq * gqq;
        }
      }
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
  for (int k = 0; k < n; ++k) {
    const int o = order[k];
    evals[k] = a(o, o).real();
    if (evecs)
      for (int i = 0; i < n; ++i) {
        evecs[2 * (i + n * k)] = v(i, o).real();
        evecs[2 * (i + n * k) + 1] = v(i, o).imag();
      }
  }
}

}  // namespace sscg
