"""Seeded synthetic inputs shared by the oracle, the GPU tests and the benchmark.

This module holds no arithmetic of the eigensolver: it only draws random SU(3)
gauge links and complex Gaussian sources, and names the workloads (lattice
sizes, hopping parameters, intervals, shift counts). Both the CPU oracle and
the HIP path receive exactly the arrays produced here.

Canonical layouts (the library's boundary layout as well):
  gauge   complex128 [4][V][3][3]   U_mu(x), row-major colour matrix; mu = 0..3
                                    is x, y, z, t; U_mu(x) multiplies psi(x+mu)
                                    in the forward hop.
  spinor  complex128 [L][V][4][3]   source index, site, spin, colour.
  site    s = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Sequence

import numpy as np


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, normalised so that Tr(l_a l_b) = 2 delta_ab."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / math.sqrt(3)
    g[7][2, 2] = -2 / math.sqrt(3)
    return g


def volume(dims: Sequence[int]) -> int:
    return int(np.prod(dims))


def gauge_field(dims: Sequence[int], eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i*eps*sum_a c_a lambda_a), c_a ~ N(0,1).

    Draw order: default_rng(seed).standard_normal((4, V, 8)) indexed [mu][s][a].
    The exponential of the Hermitian traceless generator H is taken through its
    eigen-decomposition, U = W diag(exp(i*eps*h)) W^H, so U is unitary with
    det U = exp(i*eps*Tr H) = 1 up to rounding.
    Returns complex128 [4][V][3][3].
    """
    V = volume(dims)
    c = np.random.default_rng(seed).standard_normal((4, V, 8))
    H = np.einsum("mva,aij->mvij", c, gell_mann())
    h, W = np.linalg.eigh(H)
    ph = np.exp(1j * eps * h)
    U = np.einsum("mvik,mvk,mvjk->mvij", W, ph, W.conj())
    return np.ascontiguousarray(U)


def unit_gauge(dims: Sequence[int]) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def sources(V: int, L: int, seed: int) -> np.ndarray:
    """L complex Gaussian sources, v = (a + i b)/sqrt(2), a, b ~ N(0,1).

    Draw order: default_rng([seed, 1]).standard_normal((L, 12V, 2)).
    Returns complex128 [L][V][4][3] (flattened index 12 s + 3 spin + colour).
    """
    ab = np.random.default_rng([seed, 1]).standard_normal((L, 12 * V, 2))
    v = (ab[..., 0] + 1j * ab[..., 1]) / math.sqrt(2.0)
    return np.ascontiguousarray(v.reshape(L, V, 4, 3))


def random_gauge_transform(V: int, seed: int) -> np.ndarray:
    """Random SU(3) matrix per site, complex128 [V][3][3] (for covariance checks)."""
    c = np.random.default_rng([seed, 2]).standard_normal((V, 8))
    H = np.einsum("va,aij->vij", c, gell_mann())
    h, W = np.linalg.eigh(H)
    return np.einsum("vik,vk,vjk->vij", W, np.exp(1j * h), W.conj())


@dataclass(frozen=True)
class Workload:
    """One eigensolver problem: lattice, Wilson matrix, contour and solver settings.

    The interval searched is [gamma - rho, gamma + rho]; the quadrature nodes lie on
    two horizontal lines at imaginary part +-beta*rho; the seed shift of the
    shifted CG is the interval centre gamma.
    """
    name: str
    dims: tuple
    kappa: float
    eps: float
    seed: int
    gamma: float
    rho: float
    beta: float
    N: int          # quadrature points (shifts)
    L: int          # sources
    M: int          # moments per source
    tol: float = 1e-12
    prec: str = "fp64"          # "fp64" or "mixed"
    link_reals: int = 18        # 18 or 12 (two-row SU(3) storage)
    ru_interval: int = 50
    switch_tol: float = 1e-6
    r: float = 1.0              # Wilson parameter

    @property
    def V(self) -> int:
        return volume(self.dims)

    @property
    def n(self) -> int:
        return 12 * self.V

    def gauge(self) -> np.ndarray:
        return gauge_field(self.dims, self.eps, self.seed)

    def sources(self) -> np.ndarray:
        return sources(self.V, self.L, self.seed)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The workloads: lattice 4^4 ... 24^3x48 with random SU(3) links. Where the
# problem statement leaves a value open (line offset, interval, moment count,
# tolerance) the value chosen is recorded here.
CONFIGS = {
    "wilson4_fp64": Workload("wilson4_fp64", (4, 4, 4, 4), 0.12, 0.3, 0,
                             0.0, 0.2, 0.25, 16, 1, 8),
    "wilson8_fp64": Workload("wilson8_fp64", (8, 8, 8, 8), 0.125, 0.5, 1,
                             0.0, 0.1, 0.25, 32, 4, 16),
    "wilson16x32_mixed": Workload("wilson16x32_mixed", (16, 16, 16, 32), 0.13, 0.6, 2,
                                  0.0, 0.05, 0.25, 32, 8, 16, prec="mixed"),
    "batch_8": Workload("batch_8", (8, 8, 8, 8), 0.12, 0.5, 3,
                        0.0, 0.1, 0.25, 24, 4, 12, prec="mixed"),
    "batch_12": Workload("batch_12", (12, 12, 12, 12), 0.125, 0.5, 4,
                         0.0, 0.08, 0.25, 32, 4, 16, prec="mixed"),
    "batch_16": Workload("batch_16", (16, 16, 16, 16), 0.13, 0.5, 5,
                         0.0, 0.05, 0.25, 48, 4, 24, prec="mixed"),
    "wilson24x48": Workload("wilson24x48", (24, 24, 24, 48), 0.135, 0.7, 6,
                                    0.0, 0.05, 0.4, 64, 8, 24, prec="mixed", link_reals=12),
}
BATCH = ("batch_8", "batch_12", "batch_16")
