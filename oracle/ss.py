"""Sakurai-Sugiura moments and eigenpair extraction (oracle; test infrastructure only).

Moments eq. (2):   s_k = sum_j w_j zeta_j^k y_j,  y_j = (z_j I - A)^{-1} v,  k < M,
block form with L sources (end of Sec. 2.1): S_hat = [s_{0,1..L}, ..., s_{M-1,1..L}],
an n x (M L) matrix ordered moment-major (column k L + l).

Rayleigh-Ritz (Sec. 2.1): Q = orthonormal basis of S_hat, A~ = Q^H A Q,
x = Q w, Ritz values = eigenvalues of A~ (B~ = Q^H Q = I for an orthonormal Q).
Hankel (Sec. 2.1): mu_k = V^H s_k, H = [mu_{i+j}], H< = [mu_{i+j+1}] (blocks of L x L),
eigenvalues of the pencil (H<, H) are the normalised eta = (lambda - gamma)/rho,
eigenvectors x = S_hat u.

Readings where the paper is silent:
  * Numerical rank (the paper's m is unknown): columns of S_hat are scaled to unit
    norm, and the left singular vectors with sigma_i > rank_tol * sigma_1 span Q.
    The Hankel pencil is reduced on the singular vectors of H with
    sigma_i > rank_tol * sigma_1.
  * Acceptance (Sec. 3): a pair is reported when Re lambda lies in the rectangle
    spanned by the Nprime nodes nearest gamma, |Im lambda| < beta rho, and its
    residual ||A x - lambda x|| (||x|| = 1) is at most spur_tol.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as quad
from .solvers import shifted_cg


def moments(Y: np.ndarray, zeta: np.ndarray, w: np.ndarray, M: int) -> np.ndarray:
    """Eq. (2) for every source. Y: [L][N][n] -> S: [L][M][n]."""
    c = quad.moment_coefficients(zeta, w, M)          # [M][N]
    return np.einsum("kj,ljn->lkn", c, Y)


def s_hat(S: np.ndarray) -> np.ndarray:
    """[L][M][n] -> n x (M L), column k L + l = s_{k,l}."""
    L, M, n = S.shape
    return S.transpose(2, 1, 0).reshape(n, M * L)


def orthonormal_basis(Sh: np.ndarray, rank_tol: float) -> np.ndarray:
    Sn = Sh / np.linalg.norm(Sh, axis=0)
    U, sv, _ = np.linalg.svd(Sn, full_matrices=False)
    r = int(np.sum(sv > rank_tol * sv[0]))
    return U[:, :r]


def rayleigh_ritz(Sh: np.ndarray, A_mul_cols, rank_tol: float = 1e-10):
    """Ritz pairs on span(S_hat). A_mul_cols(X) applies A to the columns of X.
    Returns (theta [r], X [n][r] unit columns, res [r])."""
    Q = orthonormal_basis(Sh, rank_tol)
    AQ = A_mul_cols(Q)
    At = Q.conj().T @ AQ
    theta, W = np.linalg.eigh(At)
    X = Q @ W
    res = np.linalg.norm(AQ @ W - X * theta[None, :], axis=0)
    return theta, X, res


def block_moments(Y: np.ndarray, Vsrc: np.ndarray, zeta, w, K: int) -> np.ndarray:
    """mu_k = V^H s_k, an L x L block per k < K. Y: [L][N][n], Vsrc: [L][n] -> [K][L][L]."""
    c = np.array([w * zeta ** k for k in range(K)])   # [K][N]
    G = np.einsum("an,bjn->jab", Vsrc.conj(), Y)       # (V^H y_j)[a][b], [N][L][L]
    return np.einsum("kj,jab->kab", c, G)


def hankel(mu: np.ndarray, Sh: np.ndarray, A_mul_cols, gamma: float, rho: float,
           M: int, rank_tol: float = 1e-10):
    """Block Hankel extraction. mu: [2M][L][L]. Returns (lambda complex [r], X, res)."""
    L = mu.shape[1]
    H = np.zeros((M * L, M * L), dtype=np.complex128)
    Hs = np.zeros_like(H)
    for i in range(M):
        for j in range(M):
            H[i * L:(i + 1) * L, j * L:(j + 1) * L] = mu[i + j]
            Hs[i * L:(i + 1) * L, j * L:(j + 1) * L] = mu[i + j + 1]
    U, sv, Wh = np.linalg.svd(H)
    r = int(np.sum(sv > rank_tol * sv[0]))
    Ur, Wr, isq = U[:, :r], Wh[:r].conj().T, 1.0 / np.sqrt(sv[:r])
    red = isq[:, None] * (Ur.conj().T @ Hs @ Wr) * isq[None, :]
    eta, T = np.linalg.eig(red)
    lam = gamma + rho * eta
    X = Sh @ (Wr @ (isq[:, None] * T))
    X = X / np.linalg.norm(X, axis=0)
    AX = A_mul_cols(X)
    res = np.linalg.norm(AX - X * lam[None, :], axis=0)
    return lam, X, res


def accept(lam, res, lo: float, hi: float, imag_max: float, spur_tol: float):
    """Indices of reported pairs (acceptance rectangle and residual filter), sorted by Re lambda."""
    lam = np.asarray(lam)
    keep = (lam.real >= lo) & (lam.real <= hi) & (np.abs(lam.imag) < imag_max) & (res <= spur_tol)
    idx = np.nonzero(keep)[0]
    return idx[np.argsort(lam.real[idx])]


def lowest_magnitude_eigs(A, k: int, tol: float = 1e-12):
    """The k eigenvalues of A of smallest magnitude with unit eigenvectors (plain
    definition of the reference spectrum on lattices too large for a dense eigh):
    Lanczos (scipy eigsh) for the smallest eigenvalues of A^2, signs and values from
    the Rayleigh quotients. Returns (lam ascending, X [n][k])."""
    import scipy.sparse.linalg as sla
    op = sla.LinearOperator(A.shape, matvec=lambda x: A @ (A @ x), dtype=np.complex128)
    _, vecs = sla.eigsh(op, k=k, which="SA", tol=tol, ncv=max(4 * k, 40))
    # the eigenspaces of A^2 mix +-lambda pairs only if both signs occur with equal
    # magnitude; a Rayleigh-Ritz step on the k-dimensional space separates them
    Q, _ = np.linalg.qr(vecs)
    lam, W = np.linalg.eigh(Q.conj().T @ (A @ Q))
    return lam, Q @ W


def weighted_tol_scale(coefs) -> np.ndarray:
    """Per-node tolerance multipliers for moment-weighted stopping.

    coefs: one [M][N_nodes] coefficient array c[k][j] = w_j zeta_j^k per pair (zero
    where a node is not in the pair). The moments use y_j only through c[k][j] y_j,
    so an error e_j in y_j enters them as |c[k][j]| e_j. Node j may stop at
    tol * m / m_j with m_j = max over pairs and k of |c[k][j]| and m = max_j m_j: its
    contribution then carries no more error than the largest-weight node at tol.
    (Nodes with m_j below 1e-12 m take the factor 1e12.)
    """
    m_j = np.max([np.abs(c).max(axis=0) for c in coefs], axis=0)
    m = m_j.max()
    return np.where(m_j > 1e-12 * m, m / np.maximum(m_j, 1e-300), 1e12)


def ss_eigs(A, Vsrc: np.ndarray, gamma: float, rho: float, beta: float, N: int, M: int,
            tol: float = 1e-12, method: str = "rr", path: str = "lines", Nprime: int | None = None,
            rank_tol: float = 1e-10, spur_tol: float = 1e-6, maxiter: int = 100000,
            weighted_tol: bool = False):
    """Full pipeline: quadrature, shifted CG per source, moments, extraction, acceptance.

    A: scipy sparse (or anything with @). Vsrc: [L][n]. Returns a dict with the
    accepted eigenvalues, unit eigenvectors (columns), residuals, and the
    intermediate quantities. weighted_tol: per-node stopping tolerances from
    weighted_tol_scale (the shifted CG then stops each node by its moment weight).
    """
    if path == "lines":
        z, zeta = quad.line_nodes(N, gamma, rho, beta)
        w = quad.line_weights(zeta)
        lo, hi = quad.acceptance_interval(zeta, gamma, rho, Nprime or N)
        imag_max = beta * rho
    elif path == "circle":
        z, zeta = quad.circle_nodes(N, gamma, rho)
        w = quad.circle_weights(zeta)
        lo, hi, imag_max = gamma - rho, gamma + rho, rho
    else:
        raise ValueError(path)
    A_mul = lambda x: A @ x
    ts = weighted_tol_scale([quad.moment_coefficients(zeta, w, M)]) if weighted_tol else None
    runs = [shifted_cg(A_mul, v, z, gamma, tol, maxiter, tol_scale=ts) for v in Vsrc]
    Y = np.array([r.Y for r in runs])
    S = moments(Y, zeta, w, M)
    Sh = s_hat(S)
    A_cols = lambda X: A @ X
    if method == "rr":
        lam, X, res = rayleigh_ritz(Sh, A_cols, rank_tol)
    elif method == "hankel":
        mu = block_moments(Y, Vsrc, zeta, w, 2 * M)
        lam, X, res = hankel(mu, Sh, A_cols, gamma, rho, M, rank_tol)
    else:
        raise ValueError(method)
    idx = accept(lam, res, lo, hi, imag_max, spur_tol)
    return dict(lam=lam[idx], X=X[:, idx], res=res[idx], all_lam=lam, all_res=res,
                z=z, zeta=zeta, w=w, Y=Y, S=S, runs=runs, lo=lo, hi=hi)


def ss_eigs_adjacent(A, Vsrc: np.ndarray, gamma: float, rho: float, beta: float, N: int, M: int,
                     Nprime: int, P: int, tol: float = 1e-12, rank_tol: float = 1e-10,
                     spur_tol: float = 1e-6, maxiter: int = 100000, weighted_tol: bool = False):
    """P adjacent line pairs sharing nodes (Sec. 3): one shifted CG over the distinct nodes,
    then per pair the moments eq. (2) over its own N nodes, Rayleigh-Ritz, and acceptance in
    its N' rectangle (half-open [lo, hi) except for the last pair, so an eigenvalue on a
    shared edge is reported once)."""
    z_all, offsets, centres = quad.adjacent_pairs(N, Nprime, P, gamma, rho, beta)
    _, zeta = quad.line_nodes(N, 0.0, 1.0, beta)
    w = quad.line_weights(zeta)
    A_mul = lambda x: A @ x
    ts = None
    if weighted_tol:
        c = quad.moment_coefficients(zeta, w, M)
        per_pair = []
        for p in range(P):
            cp = np.zeros((M, z_all.size), dtype=np.complex128)
            cp[:, offsets[p]:offsets[p] + N] = c
            per_pair.append(cp)
        ts = weighted_tol_scale(per_pair)
    runs = [shifted_cg(A_mul, v, z_all, gamma, tol, maxiter, tol_scale=ts) for v in Vsrc]
    Y_all = np.array([r.Y for r in runs])
    lams, Xs, ress = [], [], []
    for p in range(P):
        Y = Y_all[:, offsets[p]:offsets[p] + N]
        Sh = s_hat(moments(Y, zeta, w, M))
        lam, X, res = rayleigh_ritz(Sh, lambda X: A @ X, rank_tol)
        lo, hi = quad.acceptance_interval(zeta, centres[p], rho, Nprime)
        keep = (lam >= lo) & ((lam < hi) if p < P - 1 else (lam <= hi)) & (res <= spur_tol)
        lams.append(lam[keep])
        Xs.append(X[:, keep])
        ress.append(res[keep])
    lam = np.concatenate(lams)
    order = np.argsort(lam)
    return dict(lam=lam[order], X=np.concatenate(Xs, axis=1)[:, order], res=np.concatenate(ress)[order],
                z_all=z_all, offsets=offsets, centres=centres, runs=runs)
