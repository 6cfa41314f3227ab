// Host-only numerical helpers of the sscg library (no HIP types): quadrature,
// Cholesky, and the dense Hermitian eigensolver. Shared by api.cpp and the host
// sanitizer build.
#pragma once
#include <complex>
#include <vector>

namespace sscg {
using cd = std::complex<double>;
// nodes z = gamma + rho zeta, normalised nodes zeta and weights w on the two lines
// Im zeta = +-beta (Sec. 3) or on the circle |zeta| = 1 (Sec. 2.1)
void quad_lines_host(int N, double gamma, double rho, double beta, std::vector<cd> &z, std::vector<cd> &zeta,
                     std::vector<cd> &w);
void quad_circle_host(int N, double gamma, double rho, std::vector<cd> &z, std::vector<cd> &zeta, std::vector<cd> &w);
// upper Cholesky factor of a Hermitian positive definite row-major matrix and its
// inverse; false if a pivot is not positive
bool chol_inverse_upper(int n, const std::vector<cd> &G, std::vector<cd> &Rinv);
// Hermitian eigen-decomposition (dense_host.cpp); false if not converged
bool herm_eig(int n, const double *A, double *evals, double *evecs);
}  // namespace sscg
