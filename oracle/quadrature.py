"""Quadrature nodes and weights for the contour integral (oracle; test infrastructure only).

Notation of the paper: z_j are the quadrature points, zeta_j = (z_j - gamma)/rho
the normalised points (Sec. 2.1, after eq. 2), w_j the weights, and
f_k(x) = sum_j w_j zeta_j^k / (zeta_j - x) the filter function (eq. 3).

Readings taken where the paper is silent:
  * Line nodes (Sec. 3): the N/2 points of each line are equally spaced with both
    endpoints included, x_i = -1 + 2 i/(N/2 - 1); even j lie on the upper line
    (zeta = x_i + i beta), odd j on the lower one (zeta = x_i - i beta), so
    zeta_{2i+1} = conj(zeta_{2i}).
  * Weights are dimensionless for both paths: on the circle w_j = zeta_j / N (the
    paper's (z_j - gamma)/N carries an extra factor rho, a global scale that does
    not change any eigenpair).
"""
from __future__ import annotations

import numpy as np


def line_nodes(N: int, gamma: float, rho: float, beta: float):
    """Nodes on the two horizontal lines L+- (Sec. 3). Returns (z, zeta) complex [N]."""
    if N < 4 or N % 2:
        raise ValueError("N must be even and >= 4")
    h = N // 2
    x = -1.0 + 2.0 * np.arange(h) / (h - 1)
    zeta = np.empty(N, dtype=np.complex128)
    zeta[0::2] = x + 1j * beta
    zeta[1::2] = x - 1j * beta
    return gamma + rho * zeta, zeta


def line_weights(zeta: np.ndarray) -> np.ndarray:
    """Weights solving sum_j w_j zeta_j^(k-1) = delta_k0, k = 0..N-1 (Sec. 3).

    The system asks w to annihilate every polynomial of degree <= N-2 at the nodes
    and to give 1 for 1/zeta. The first condition makes w_j proportional to
    1/prod_{i != j}(zeta_j - zeta_i) (the divided-difference weights); the divided
    difference of 1/x over all nodes is (-1)^(N-1)/prod_i zeta_i, which fixes the
    constant. Written out:  w_j = zeta_j prod_{i != j} zeta_i / (zeta_i - zeta_j).
    (A direct FP64 Vandermonde solve is useless here: its condition number passes
    1e17 at N = 64.)
    """
    N = zeta.size
    w = np.empty(N, dtype=np.complex128)
    for j in range(N):
        others = np.delete(zeta, j)
        w[j] = zeta[j] * np.prod(others / (others - zeta[j]))
    return w


def circle_nodes(N: int, gamma: float, rho: float):
    """Circle C of centre gamma and radius rho (Sec. 2.1): z_j = gamma + rho e^{2 pi i (j+1/2)/N}."""
    zeta = np.exp(2j * np.pi * (np.arange(N) + 0.5) / N)
    return gamma + rho * zeta, zeta


def circle_weights(zeta: np.ndarray) -> np.ndarray:
    """Circle weights (Sec. 2.1), dimensionless: w_j = zeta_j / N."""
    return zeta / zeta.size


def filter_function(x, zeta: np.ndarray, w: np.ndarray, k: int = 0):
    """f_k(x) = sum_j w_j zeta_j^k / (zeta_j - x), eq. (3)."""
    x = np.asarray(x, dtype=np.complex128)
    return np.sum((w * zeta ** k)[:, None] / (zeta[:, None] - x.ravel()[None, :]), axis=0).reshape(x.shape)


def moment_coefficients(zeta: np.ndarray, w: np.ndarray, M: int) -> np.ndarray:
    """c[k][j] = w_j zeta_j^k for k < M: the coefficients of eq. (2)."""
    return np.array([w * zeta ** k for k in range(M)])


def acceptance_interval(zeta: np.ndarray, gamma: float, rho: float, Nprime: int):
    """Real range of the rectangle formed by the Nprime nodes nearest gamma (Sec. 3).

    The line nodes come in conjugate pairs; the Nprime/2 pairs whose real parts are
    closest to the centre span the rectangle. Returns (lo, hi) in z units.
    """
    if Nprime < 4 or Nprime % 2:
        raise ValueError("Nprime must be even and >= 4")
    xr = np.unique(np.round(zeta.real, 14))
    if Nprime // 2 > xr.size:
        raise ValueError("Nprime larger than the node count")
    order = np.argsort(np.abs(xr))[: Nprime // 2]
    sel = np.sort(xr[order])
    return gamma + rho * sel[0], gamma + rho * sel[-1]


def adjacent_pairs(N: int, Nprime: int, P: int, gamma: float, rho: float, beta: float):
    """P line pairs side by side with shared nodes (Sec. 3, last paragraph).

    Every pair has N nodes, half-width rho and offset beta; pair p + 1 is pair p moved
    right by the N'-2 nodes (N'/2 - 1 per line) that span its acceptance rectangle,
    so the rectangles tile [first lo, last hi] and each new pair adds N' - 2 nodes.
    The pairs are centred on gamma as a group. Returns
      z_all [N + (P-1)(N'-2)]  distinct nodes, ordered as in line_nodes (even index on
                               the upper line) along the common grid,
      offsets [P]              pair p uses z_all[offsets[p] : offsets[p] + N],
      centres [P]              the pair centres gamma_p,
    and the per-pair normalised nodes are those of line_nodes(N, 0, 1, beta).
    """
    if Nprime < 4 or Nprime % 2 or Nprime > N:
        raise ValueError("need even 4 <= Nprime <= N")
    h = 2.0 * rho / (N // 2 - 1)          # node spacing along a line
    step = (Nprime - 2) // 2              # nodes per line between neighbouring pairs
    total_x = N // 2 + (P - 1) * step
    span = (P - 1) * step * h             # distance between the first and last centre
    x = (gamma - 0.5 * span - rho) + h * np.arange(total_x)
    z_all = np.empty(2 * total_x, dtype=np.complex128)
    z_all[0::2] = x + 1j * beta * rho
    z_all[1::2] = x - 1j * beta * rho
    offsets = 2 * step * np.arange(P)
    centres = gamma - 0.5 * span + step * h * np.arange(P)
    return z_all, offsets, centres
