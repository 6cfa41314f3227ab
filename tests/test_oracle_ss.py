"""Pins of the oracle's moments eq. (2), Rayleigh-Ritz and Hankel extraction (Sec. 2.1)
and acceptance (Sec. 3).

* An eigenvector source v = x_l gives s_k = f_k(eta_l)/rho x_l exactly (Sec. 2.1,
  after eq. 3), with f_k from the filter's product form; the Hankel pencil of one
  or two modes returns their eta exactly.
* Rayleigh-Ritz on a window of the 4^4 field reproduces the dense spectrum.
* Eigenvalues outside the contour never appear (free field, closed-form spectrum);
  inside, a degenerate eigenvalue is recovered min(L, multiplicity) times.
* The specified 4^4 workload has no eigenvalue in [-0.2, 0.2]: the output is empty.
* Every reported pair is certified by its residual (Hermitian A).
"""
import numpy as np
import pytest

import synth
from oracle import quadrature as quad
from oracle import ss, wilson

CFG1 = synth.CONFIGS["wilson4_fp64"]


@pytest.fixture(scope="module")
def spec(cfg1_dense):
    U, A, lam, W = cfg1_dense
    return A, lam, W


def product_filter(x, zeta):
    return np.prod(zeta / (zeta - x))


def test_moments_of_an_eigenvector_source(spec):
    A, lam, W = spec
    gamma, rho, beta, N, M = 0.2, 0.05, 0.3, 16, 6
    l = np.argmin(np.abs(lam - 0.21))
    x = W[:, l]
    z, zeta = quad.line_nodes(N, gamma, rho, beta)
    w = quad.line_weights(zeta)
    Y = np.array([[x / (zj - lam[l]) for zj in z]])       # exact solves
    S = ss.moments(Y, zeta, w, M)
    eta = (lam[l] - gamma) / rho
    for k in range(M):
        fk = eta ** k * product_filter(eta, zeta)
        assert np.linalg.norm(S[0, k] - fk / rho * x) < 1e-12 * max(1, abs(fk) / rho)


def test_hankel_recovers_single_and_double_modes(spec):
    A, lam, W = spec
    gamma, rho, beta, N = 0.225, 0.03, 0.25, 16
    z, zeta = quad.line_nodes(N, gamma, rho, beta)
    w = quad.line_weights(zeta)
    idx = np.argsort(np.abs(lam - gamma))[:2]
    for modes, M in (([idx[0]], 1), (list(idx), 2)):
        v = W[:, modes].sum(axis=1)
        Y = np.array([[W[:, modes] @ ((W[:, modes].conj().T @ v) / (zj - lam[modes])) for zj in z]])
        mu = ss.block_moments(Y, v[None, :], zeta, w, 2 * M)
        Sh = ss.s_hat(ss.moments(Y, zeta, w, M))
        got, X, res = ss.hankel(mu, Sh, lambda X: A @ X, gamma, rho, M, rank_tol=1e-12)
        assert np.allclose(np.sort(got.real), np.sort(lam[modes]), atol=1e-13, rtol=0)
        assert np.abs(got.imag).max() < 1e-13
        assert res.max() < 1e-12


def test_rayleigh_ritz_window_matches_dense_spectrum(spec):
    A, lam, W = spec
    w = CFG1.with_(gamma=0.225, rho=0.03, L=2)
    V = synth.sources(w.V, w.L, w.seed).reshape(w.L, -1)
    out = ss.ss_eigs(A, V, w.gamma, w.rho, w.beta, w.N, w.M, rank_tol=1e-7)
    truth = lam[(lam >= w.gamma - w.rho) & (lam <= w.gamma + w.rho)]
    assert len(out["lam"]) == len(truth) == 6
    assert np.abs(out["lam"] - truth).max() < 1e-10 * 0.225
    assert out["res"].max() < 1e-8


@pytest.mark.parametrize("method", ["rr", "hankel"])
def test_reported_pairs_are_certified_by_residual(spec, method):
    A, lam, W = spec
    w = CFG1.with_(gamma=0.225, rho=0.03, L=2)
    V = synth.sources(w.V, w.L, w.seed).reshape(w.L, -1)
    out = ss.ss_eigs(A, V, w.gamma, w.rho, w.beta, w.N, w.M, method=method, rank_tol=1e-7)
    assert len(out["lam"]) > 0
    for l, r in zip(out["lam"].real, out["res"]):
        assert np.abs(lam - l).min() <= r + 1e-14
    for i, x in enumerate(out["X"].T):
        assert abs(np.linalg.norm(x) - 1) < 1e-12


def test_specified_4444_workload_is_empty(spec):
    A, lam, W = spec
    assert np.sum(np.abs(lam - CFG1.gamma) <= CFG1.rho) == 0
    assert np.min(np.abs(lam)) == pytest.approx(0.2191, abs=1e-4)
    V = CFG1.sources().reshape(CFG1.L, -1)
    for method in ("rr", "hankel"):
        out = ss.ss_eigs(A, V, CFG1.gamma, CFG1.rho, CFG1.beta, CFG1.N, CFG1.M, method=method)
        assert len(out["lam"]) == 0


@pytest.mark.parametrize("L", [1, 2, 7])
def test_free_field_outside_never_appears(L):
    dims, kappa = (4, 4, 4, 4), 0.12
    A = wilson.hermitian_wilson(synth.unit_gauge(dims), dims, kappa)
    V = synth.sources(256, L, 3).reshape(L, -1)
    out = ss.ss_eigs(A, V, 0.0, 0.03, 0.25, 16, 8)
    assert len(out["lam"]) == 0
    out = ss.ss_eigs(A, V, 0.0, 0.05, 0.25, 16, 8)
    got = np.sort(out["lam"].real)
    m = min(L, 6)
    assert len(got) == 2 * m
    assert np.allclose(got, [-0.04] * m + [0.04] * m, atol=1e-12)


def test_moments_are_linear_in_the_solutions():
    rng = np.random.default_rng(0)
    N, M, n = 16, 5, 50
    _, zeta = quad.line_nodes(N, 0.0, 1.0, 0.3)
    w = quad.line_weights(zeta)
    Y1 = rng.standard_normal((2, N, n)) + 1j * rng.standard_normal((2, N, n))
    Y2 = rng.standard_normal((2, N, n)) + 1j * rng.standard_normal((2, N, n))
    a = 0.3 - 1.2j
    lhs = ss.moments(Y1 + a * Y2, zeta, w, M)
    rhs = ss.moments(Y1, zeta, w, M) + a * ss.moments(Y2, zeta, w, M)
    assert np.abs(lhs - rhs).max() < 1e-12
    # the k-th moment of a single node's unit vector is w_j zeta_j^k
    E = np.zeros((1, N, 1), dtype=complex)
    E[0, 3, 0] = 1
    assert np.allclose(ss.moments(E, zeta, w, M)[0, :, 0], w[3] * zeta[3] ** np.arange(M))


def test_lowest_magnitude_eigs_matches_dense():
    dims = (3, 3, 3, 3)
    A = wilson.hermitian_wilson(synth.gauge_field(dims, 0.5, 2), dims, 0.13)
    lam = np.linalg.eigvalsh(A.toarray())
    got, X = ss.lowest_magnitude_eigs(A, 12)
    ref = np.sort(lam[np.argsort(np.abs(lam))[:12]])
    assert np.abs(got - ref).max() < 1e-12
    assert np.linalg.norm(A @ X - X * got[None, :], axis=0).max() < 1e-9


def test_adjacent_pairs_equal_separate_runs(spec):
    """Three adjacent pairs over [0.205, 0.245] on the 4^4 field give, pair by pair, the
    same accepted eigenvalues as three separate single-pair runs (Sec. 3)."""
    A, lam, W = spec
    V = synth.sources(CFG1.V, 2, 5).reshape(2, -1)
    N, Np, P, rho, beta, M = 16, 8, 3, 0.012, 0.25, 6
    out = ss.ss_eigs_adjacent(A, V, 0.225, rho, beta, N, M, Np, P, rank_tol=1e-7)
    sep = []
    for p, c in enumerate(out["centres"]):
        o = ss.ss_eigs(A, V, c, rho, beta, N, M, Nprime=Np, rank_tol=1e-7)
        _, zeta = quad.line_nodes(N, 0.0, 1.0, beta)
        lo, hi = quad.acceptance_interval(zeta, c, rho, Np)
        keep = (o["lam"] >= lo) & ((o["lam"] < hi) if p < P - 1 else (o["lam"] <= hi))
        sep.extend(o["lam"][keep])
    assert len(out["lam"]) == len(sep) > 0
    assert np.abs(np.sort(out["lam"]) - np.sort(sep)).max() < 1e-12
    lo_all = out["centres"][0] - rho * (Np // 2 - 1) / (N // 2 - 1)
    hi_all = out["centres"][-1] + rho * (Np // 2 - 1) / (N // 2 - 1)
    truth = lam[(lam >= lo_all) & (lam <= hi_all)]
    assert np.abs(np.sort(out["lam"]) - truth).max() < 1e-10


def test_weighted_tolerance_keeps_the_moments(spec):
    """Moment-weighted stopping (each node stops at tol * m / m_j): fewer shift updates,
    the moments stay within a few times the uniform-tolerance error of the exact
    moments from dense spectral solves, and the eigenpairs are unchanged."""
    A, lam, W = spec
    V = synth.sources(CFG1.V, 2, 9).reshape(2, -1)
    gamma, rho, beta, N, M = 0.225, 0.03, 0.25, 16, 8
    z, zeta = quad.line_nodes(N, gamma, rho, beta)
    w = quad.line_weights(zeta)
    c = quad.moment_coefficients(zeta, w, M)
    ts = ss.weighted_tol_scale([c])
    m_j = np.abs(c).max(axis=0)
    assert np.allclose(ts * m_j, m_j.max()) and ts.min() == 1.0
    Yx = np.array([[W @ ((W.conj().T @ v) / (zj - lam)) for zj in z] for v in V])
    Sx = ss.moments(Yx, zeta, w, M)
    u = ss.ss_eigs(A, V, gamma, rho, beta, N, M, rank_tol=1e-7)
    g = ss.ss_eigs(A, V, gamma, rho, beta, N, M, rank_tol=1e-7, weighted_tol=True)
    su = lambda out: sum(int(np.where(r.conv_iter >= 0, r.conv_iter, r.iters).sum()) for r in out["runs"])
    assert su(g) < su(u)
    eu = np.abs(u["S"] - Sx).max()
    eg = np.abs(g["S"] - Sx).max()
    assert eg <= 10 * max(eu, 1e-13 * np.abs(Sx).max())
    assert len(g["lam"]) == len(u["lam"]) > 0
    assert np.all(np.abs(g["lam"] - u["lam"]) <= 1e-10 * np.abs(u["lam"]))
    assert g["res"].max() < 1e-8
