// Host FP64 helpers with no device code: quadrature nodes and weights on the two
// lines (Sec. 3) and the circle (Sec. 2.1), and the Cholesky factor used by the
// Rayleigh-Ritz orthogonalisation (Sec. 2.1). Built as plain C++ (also by the
// sanitizer test of the host code).
#include <cmath>
#include <complex>
#include <vector>

#include "host_math.h"

namespace sscg {

void quad_lines_host(int N, double gamma, double rho, double beta, std::vector<cd> &z, std::vector<cd> &zeta,
                            std::vector<cd> &w) {
  const int h = N / 2;
  z.resize(N);
  zeta.resize(N);
  w.resize(N);
  for (int i = 0; i < h; ++i) {
    const double x = -1.0 + 2.0 * i / (h - 1);
    zeta[2 * i] = cd(x, beta);
    zeta[2 * i + 1] = cd(x, -beta);
  }
  // w_j = zeta_j prod_{i != j} zeta_i / (zeta_i - zeta_j): the unique solution of
  // sum_j w_j zeta_j^(k-1) = delta_k0, k < N (Lagrange / divided-difference form).
  for (int j = 0; j < N; ++j) {
    cd prod = zeta[j];
    for (int i = 0; i < N; ++i)
      if (i != j) prod *= zeta[i] / (zeta[i] - zeta[j]);
    w[j] = prod;
    z[j] = gamma + rho * zeta[j];
  }
}
void quad_circle_host(int N, double gamma, double rho, std::vector<cd> &z, std::vector<cd> &zeta,
                             std::vector<cd> &w) {
  z.resize(N);
  zeta.resize(N);
  w.resize(N);
  for (int j = 0; j < N; ++j) {
    const double th = 2.0 * M_PI * (j + 0.5) / N;
    zeta[j] = cd(std::cos(th), std::sin(th));
    z[j] = gamma + rho * zeta[j];
    w[j] = zeta[j] / (double)N;
  }
}


// Upper Cholesky factor of a Hermitian positive definite row-major n x n matrix,
// G = R^H R, and its inverse Rinv (row-major, upper triangular). Returns false if a
// pivot is not positive.
bool chol_inverse_upper(int n, const std::vector<cd> &G, std::vector<cd> &Rinv) {
  std::vector<cd> R((size_t)n * n, cd(0, 0));
  for (int j = 0; j < n; ++j) {
    double d = G[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(R[(size_t)k * n + j]);
    if (!(d > 0.0)) return false;
    const double rjj = std::sqrt(d);
    R[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) {
      cd v = G[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) v -= std::conj(R[(size_t)k * n + j]) * R[(size_t)k * n + i];
      R[(size_t)j * n + i] = v / rjj;
    }
  }
  Rinv.assign((size_t)n * n, cd(0, 0));
  for (int i = 0; i < n; ++i) {  // column i of R^-1 by back substitution
    Rinv[(size_t)i * n + i] = 1.0 / R[(size_t)i * n + i];
    for (int j = i - 1; j >= 0; --j) {
      cd v = 0;
      for (int k = j + 1; k <= i; ++k) v += R[(size_t)j * n + k] * Rinv[(size_t)k * n + i];
      Rinv[(size_t)j * n + i] = -v / R[(size_t)j * n + j];
    }
  }
  return true;
}

}  // namespace sscg
