"""Explicit Hermitian Wilson fermion matrix (oracle; test infrastructure only).

The paper (Sec. 4) defines A = gamma5 (I - kappa D) with D the Wilson hopping
matrix, which it only cites. Reading used here (standard Wilson, parameter r):

    (D psi)(x) = sum_mu [ (r - gamma_mu) U_mu(x) psi(x + mu)
                        + (r + gamma_mu) U_mu(x - mu)^H psi(x - mu) ]

with periodic boundaries in all four directions, Euclidean Dirac matrices in the
chiral basis (gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1)) and
vector index 12 s + 3 spin + colour. The matrix is assembled entry by entry as
a scipy CSR matrix from Kronecker products of 4x4 spin and 3x3 colour blocks,
which is the plain definition written out (no spin projection tricks).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def gamma_matrices() -> np.ndarray:
    """[gamma1, gamma2, gamma3, gamma4, gamma5] in the chiral (DeGrand-Rossi) basis."""
    i = 1j
    g = np.zeros((5, 4, 4), dtype=np.complex128)
    g[0] = [[0, 0, 0, i], [0, 0, i, 0], [0, -i, 0, 0], [-i, 0, 0, 0]]
    g[1] = [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]]
    g[2] = [[0, 0, i, 0], [0, 0, 0, -i], [-i, 0, 0, 0], [0, i, 0, 0]]
    g[3] = [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]]
    g[4] = g[0] @ g[1] @ g[2] @ g[3]
    return g


def coords(dims):
    """Site coordinates [V][4] for s = x + Lx (y + Ly (z + Lz t))."""
    V = int(np.prod(dims))
    s = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = s % dims[mu]
        s = s // dims[mu]
    return out


def site_index(c, dims):
    s = np.zeros(c.shape[0], dtype=np.int64)
    for mu in reversed(range(4)):
        s = s * dims[mu] + c[:, mu]
    return s


def neighbour(dims, mu: int, step: int) -> np.ndarray:
    """Periodic neighbour index array: nb[s] = s + step * mu_hat."""
    c = coords(dims)
    c[:, mu] = (c[:, mu] + step) % dims[mu]
    return site_index(c, dims)


def adjoint(M: np.ndarray) -> np.ndarray:
    """Hermitian conjugate of a stack of colour matrices [..., 3, 3]."""
    return M.conj().swapaxes(-1, -2)


def hermitian_wilson(U: np.ndarray, dims, kappa: float, r: float = 1.0) -> sp.csr_matrix:
    """A = gamma5 (I - kappa D) as an explicit sparse matrix (Sec. 4).

    U: complex128 [4][V][3][3]. Each hop contributes the 12x12 block
    -kappa * gamma5 (r -+ gamma_mu) (x) U; only the nonzero spin entries are stored,
    so every row has 1 + 8*2*3 = 49 stored entries.
    """
    V = int(np.prod(dims))
    g = gamma_matrices()
    g5 = g[4]
    I4 = np.eye(4)
    rows, cols, vals = [], [], []
    s = np.arange(V)

    def add_block(spin: np.ndarray, col_site: np.ndarray, colour: np.ndarray):
        # colour: [V][3][3]; entry (12 s + 3 a + i, 12 t + 3 b + j) = spin[a,b] colour[s,i,j]
        for a, b in itertools.product(range(4), range(4)):
            if spin[a, b] == 0:
                continue
            for ci, cj in itertools.product(range(3), range(3)):
                rows.append(12 * s + 3 * a + ci)
                cols.append(12 * col_site + 3 * b + cj)
                vals.append(spin[a, b] * colour[:, ci, cj])

    # diagonal gamma5 (x) 1: only the colour-diagonal entries are nonzero
    for a in range(4):
        for ci in range(3):
            rows.append(12 * s + 3 * a + ci)
            cols.append(12 * s + 3 * a + ci)
            vals.append(np.full(V, g5[a, a]))
    for mu in range(4):
        fwd = neighbour(dims, mu, +1)
        bwd = neighbour(dims, mu, -1)
        add_block(-kappa * (g5 @ (r * I4 - g[mu])), fwd, U[mu])
        add_block(-kappa * (g5 @ (r * I4 + g[mu])), bwd, adjoint(U[mu][bwd]))
    n = 12 * V
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def free_field_spectrum(dims, kappa: float, r: float = 1.0) -> np.ndarray:
    """Eigenvalues of A for unit links, from the plane-wave closed form.

    For momentum p_mu = 2 pi n_mu / L_mu the Wilson matrix acts as
    m + i sum_mu gamma_mu s_mu with m = 1 - 2 kappa r sum cos p_mu and
    s_mu = 2 kappa sin p_mu; A^2 = m^2 + sum s_mu^2, and A has both signs, each
    six-fold (two spin states times three colours). Returns the sorted 12V values.
    """
    ps = [2 * np.pi * np.arange(L) / L for L in dims]
    P = np.stack(np.meshgrid(*ps, indexing="ij"), axis=-1).reshape(-1, 4)
    m = 1 - 2 * kappa * r * np.cos(P).sum(1)
    lam = np.sqrt(m ** 2 + 4 * kappa ** 2 * (np.sin(P) ** 2).sum(1))
    return np.sort(np.concatenate([np.repeat(lam, 6), np.repeat(-lam, 6)]))


def to_vec(psi: np.ndarray) -> np.ndarray:
    """Canonical spinor array [..., V, 4, 3] -> flat vectors [..., 12V]."""
    return psi.reshape(psi.shape[:-3] + (-1,))


def apply_rows(U: np.ndarray, dims, kappa: float, x: np.ndarray, sites, r: float = 1.0) -> np.ndarray:
    """(A x) restricted to the 12 rows of each listed site, from the definition.

    For lattices where the explicit matrix is too large: every listed site sums its
    own term and its eight hops, each as the Kronecker product of the 4x4 spin
    factor and the 3x3 link (the same blocks as hermitian_wilson). x: [12V] or
    [V][4][3]. Returns [len(sites)][12].
    """
    g = gamma_matrices()
    g5 = g[4]
    I4 = np.eye(4)
    xv = np.asarray(x).reshape(-1, 12)
    sites = np.asarray(sites, dtype=np.int64)
    c = coords(dims)[sites]
    out = np.einsum("ab,sb->sa", np.kron(g5, np.eye(3)), xv[sites])
    for mu in range(4):
        cf = c.copy()
        cf[:, mu] = (cf[:, mu] + 1) % dims[mu]
        cb = c.copy()
        cb[:, mu] = (cb[:, mu] - 1) % dims[mu]
        fwd, bwd = site_index(cf, dims), site_index(cb, dims)
        Pf = -kappa * (g5 @ (r * I4 - g[mu]))
        Pb = -kappa * (g5 @ (r * I4 + g[mu]))
        for k in range(len(sites)):
            out[k] += np.kron(Pf, U[mu, sites[k]]) @ xv[fwd[k]]
            out[k] += np.kron(Pb, adjoint(U[mu, bwd[k]])) @ xv[bwd[k]]
    return out
