"""Pins of the oracle's shifted CG (Sec. 2.2, eq. 5 and the Hermitian-seed argument).

* Converged solutions equal the spectral solution W diag(1/(z - lambda)) W^H v from a
  dense eigen-decomposition (4^4 lattice).
* At a fixed iteration k every shifted iterate is the Galerkin (FOM) solution on the
  Krylov space K_k(A, v), computed here from an independently built Lanczos basis;
  it does not depend on the seed shift.
* One shift equal to the seed reduces to textbook CG (scipy's cg, positive definite seed).
* The implicit residual sqrt(rho)/|pi_j| equals the true shifted residual (collinearity).
* Conjugate nodes have conjugate scalars, hence identical convergence iterations.
* The independent per-shift route (CG on the normal equations of each z_j I - A)
  reaches the spectral solution of every shift.
* Failure paths: zero source, maxiter, breakdown on B v = 0, a shift on an eigenvalue.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import synth
from oracle import quadrature as quad
from oracle import solvers, wilson

CFG1 = synth.CONFIGS["wilson4_fp64"]


@pytest.fixture(scope="module")
def cfg1_spec(cfg1_dense):
    U, A, lam, W = cfg1_dense
    return A, lam, W


def spectral_solve(lam, W, z, v):
    c = W.conj().T @ v
    return np.array([W @ (c / (zj - lam)) for zj in z])


def test_converged_matches_spectral_solution(cfg1_spec):
    A, lam, W = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    r = solvers.shifted_cg(lambda x: A @ x, v, z, CFG1.gamma, 1e-12)
    assert r.status == "ok"
    Y = spectral_solve(lam, W, z, v)
    assert np.linalg.norm(r.Y - Y) / np.linalg.norm(Y) < 1e-10
    assert solvers.true_residuals(lambda x: A @ x, v, z, r.Y).max() < 2e-12


def test_normal_cg_matches_spectral_solution(cfg1_spec):
    """normal_cg, which shares nothing with the shifted recurrences, reaches the dense
    spectral solution of every node (per-shift bar: its condition number times the
    1e-13 residual it stops at is below 1e-11)."""
    A, lam, W = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    Y = solvers.normal_cg(lambda X: (A @ X.T).T, z, np.tile(v, (z.size, 1)), tol=1e-13)
    Yref = spectral_solve(lam, W, z, v)
    for j in range(z.size):
        assert np.abs(Y[j] - Yref[j]).max() <= 1e-10 * np.abs(Yref[j]).max()
    assert solvers.true_residuals(lambda x: A @ x, v, z, Y).max() < 1e-13


def test_normal_cg_pin_catches_a_conjugated_node(cfg1_spec):
    """Planted mistake: solving with conj(z_j) in place of z_j (a conjugation slip in
    B_j or B_j^H) gives another vector, which the pin above would reject."""
    A, lam, W = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    zc = np.conj(z)
    Y = solvers.normal_cg(lambda X: (A @ X.T).T, zc, np.tile(v, (z.size, 1)), tol=1e-13, maxiter=400)
    Yref = spectral_solve(lam, W, z, v)
    assert max(np.abs(Y[j] - Yref[j]).max() / np.abs(Yref[j]).max() for j in range(z.size)) > 1e-3


def lanczos_basis(A, v, k):
    """Orthonormal basis of K_k(A, v) by Lanczos with full reorthogonalisation."""
    Q = np.zeros((v.size, k), dtype=complex)
    Q[:, 0] = v / np.linalg.norm(v)
    for i in range(1, k):
        w = A @ Q[:, i - 1]
        for _ in range(2):
            w -= Q[:, :i] @ (Q[:, :i].conj().T @ w)
        Q[:, i] = w / np.linalg.norm(w)
    return Q


@pytest.mark.parametrize("sigma", [0.0, 0.07, -0.3])
def test_iterates_are_galerkin_solutions(cfg1_spec, sigma):
    A, _, _ = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    k = 12
    snap = {}

    def rec(it, st):
        if it == k - 1:
            snap["X"] = st["X"].copy()

    solvers.shifted_cg(lambda x: A @ x, v, z, sigma, 1e-30, maxiter=k, record=rec)
    Q = lanczos_basis(A, v, k)
    AQ = A @ Q
    for j, zj in enumerate(z):
        Hk = Q.conj().T @ (zj * Q - AQ)
        x = Q @ np.linalg.solve(Hk, Q.conj().T @ v)
        assert np.linalg.norm(snap["X"][j] - x) / np.linalg.norm(x) < 1e-9


def test_single_shift_at_seed_is_textbook_cg(cfg1_spec):
    A, _, _ = cfg1_spec
    v = CFG1.sources().reshape(-1)
    sigma = 2.5   # > ||A|| <= 1 + 8 kappa: the seed matrix is positive definite
    k = 15
    snap = {}

    def rec(it, st):
        if it == k - 1:
            snap["x"] = st["X"][0].copy()

    solvers.shifted_cg(lambda x: A @ x, v, np.array([sigma + 0j]), sigma, 1e-30, maxiter=k, record=rec)
    B = sla.LinearOperator(A.shape, matvec=lambda x: sigma * x - A @ x, dtype=complex)
    xs = []
    sla.cg(B, v, rtol=1e-30, atol=0.0, maxiter=k, callback=lambda xk: xs.append(xk.copy()))
    assert np.linalg.norm(snap["x"] - xs[k - 1]) / np.linalg.norm(xs[k - 1]) < 1e-12


def test_implicit_equals_true_residual(cfg1_spec):
    A, _, _ = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    snap = {}

    def rec(it, st):
        if it == 29:
            snap.update(X=st["X"].copy(), pi=st["pi"].copy(), rho=st["rho"])

    solvers.shifted_cg(lambda x: A @ x, v, z, CFG1.gamma, 1e-30, maxiter=30, record=rec)
    implicit = np.sqrt(snap["rho"]) / np.abs(snap["pi"])
    true = np.array([np.linalg.norm(v - (zj * x - A @ x)) for zj, x in zip(z, snap["X"])])
    assert np.abs(implicit - true).max() / true.max() < 1e-9


def test_conjugate_nodes_share_convergence(cfg1_spec):
    A, _, _ = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    r = solvers.shifted_cg(lambda x: A @ x, v, z, CFG1.gamma, 1e-12)
    assert np.array_equal(r.conv_iter[0::2], r.conv_iter[1::2])
    # nodes closer to the real-axis ends need more iterations (Sec. 3, Fig. 1 trend)
    assert r.conv_iter[0] >= r.conv_iter[CFG1.N // 2]


def test_zero_source_rejected(cfg1_spec):
    A, _, _ = cfg1_spec
    with pytest.raises(ValueError):
        solvers.shifted_cg(lambda x: A @ x, np.zeros(CFG1.n, complex), np.array([0.1j]), 0.0)


def test_maxiter_reports_not_converged(cfg1_spec):
    A, _, _ = cfg1_spec
    v = CFG1.sources().reshape(-1)
    r = solvers.shifted_cg(lambda x: A @ x, v, np.array([0.05j]), 0.0, 1e-12, maxiter=1)
    assert r.status == "notconv" and r.iters == 1 and r.conv_iter[0] == -1


def free_field_mode(dims):
    """Zero-momentum spinor with spin 0, colour 0: A v = (1 - 8 kappa) v for unit links.
    At kappa = 1/8 every term is a dyadic rational, so A v = 0 holds exactly."""
    V = int(np.prod(dims))
    v = np.zeros((V, 4, 3), dtype=complex)
    v[:, 0, 0] = 1.0
    return v.reshape(-1)


def test_breakdown_when_seed_annihilates_source():
    dims, kappa = (4, 4, 4, 4), 0.125
    A = wilson.hermitian_wilson(synth.unit_gauge(dims), dims, kappa)
    v = free_field_mode(dims)
    assert np.all(A @ v == 0)
    r = solvers.shifted_cg(lambda x: A @ x, v, np.array([0.01j]), 0.0, 1e-12)
    assert r.status == "breakdown" and r.iters == 0


def test_shift_on_an_eigenvalue_never_converges():
    dims, kappa = (4, 4, 4, 4), 0.12
    A = wilson.hermitian_wilson(synth.unit_gauge(dims), dims, kappa)
    v = synth.sources(256, 1, 7).reshape(-1)
    z = np.array([0.04 + 0j, 0.04 + 0.05j, -0.1 + 0.05j])
    r = solvers.shifted_cg(lambda x: A @ x, v, z, 0.0, 1e-12, maxiter=300)
    assert r.status == "notconv"
    assert r.conv_iter[0] == -1 and r.conv_iter[1] > 0 and r.conv_iter[2] > 0


def test_per_shift_tolerance(cfg1_spec):
    """tol_scale[j] moves shift j's stopping point and nothing else: each shift freezes
    at the first iteration where its implicit residual is below tol * tol_scale[j]
    ||v||, its true residual (dense spectral solve) is at that level, and the shifts
    with scale 1 are bitwise those of the unscaled run."""
    A, lam, W = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    scale = np.ones(z.size)
    scale[:4] = 1e4
    hist = []
    r1 = solvers.shifted_cg(lambda x: A @ x, v, z, CFG1.gamma, 1e-12, tol_scale=scale,
                            record=lambda k, st: hist.append(np.sqrt(st["rho"]) / np.abs(st["pi"])))
    r0 = solvers.shifted_cg(lambda x: A @ x, v, z, CFG1.gamma, 1e-12)
    assert r1.status == r0.status == "ok"
    hist = np.array(hist)
    vn = np.linalg.norm(v)
    for j in range(z.size):
        first = np.nonzero(hist[:, j] <= 1e-12 * scale[j] * vn)[0][0] + 1
        assert r1.conv_iter[j] == first
    assert np.all(r1.conv_iter[:4] < r0.conv_iter[:4])
    assert np.array_equal(r1.Y[4:], r0.Y[4:])
    Y = spectral_solve(lam, W, z, v)
    err = np.linalg.norm(r1.Y - Y, axis=1)
    res = solvers.true_residuals(lambda x: A @ x, v, z, r1.Y)
    assert np.all(res[:4] <= 1e-8 * 1.5) and np.all(res[:4] > 1e-12)
    assert np.all(res[4:] < 2e-12)
    assert np.all(err[:4] > err[4:].max())


def test_fp32_shift_emulation(cfg1_spec):
    """The FP32-shift precision schedule: never switching reproduces the FP64 run bit
    for bit; switching at 1e-6 keeps every shifted solution within 1e-10 of the dense
    spectral solution (true residual below 1e-10); switching at the start (planted
    mistake: FP32 from iteration 0) leaves errors above 1e-8, so the emulation is
    really rounding to complex64."""
    A, lam, W = cfg1_spec
    v = CFG1.sources().reshape(-1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    Amul = lambda x: A @ x
    exact = spectral_solve(lam, W, z, v)
    r64 = solvers.shifted_cg(Amul, v, z, CFG1.gamma, 1e-12)
    rnone = solvers.shifted_cg(Amul, v, z, CFG1.gamma, 1e-12, fp32_switch=0.0)
    assert np.array_equal(r64.Y, rnone.Y)
    rsw = solvers.shifted_cg(Amul, v, z, CFG1.gamma, 1e-12, fp32_switch=1e-6, fold_every=20)
    assert rsw.status == "ok"
    err = np.linalg.norm(rsw.Y - exact, axis=1) / np.linalg.norm(exact, axis=1)
    assert err.max() < 1e-10
    assert solvers.true_residuals(Amul, v, z, rsw.Y).max() < 1e-10
    assert np.abs(rsw.conv_iter - r64.conv_iter).max() <= 4
    r0 = solvers.shifted_cg(Amul, v, z, CFG1.gamma, 1e-12, fp32_switch=10.0, maxiter=2000)
    err0 = np.linalg.norm(r0.Y - exact, axis=1) / np.linalg.norm(exact, axis=1)
    assert err0.max() > 1e-8


def test_golden_wilson8_certified_by_normal_equations():
    """The stored 8^4 shifted-CG solutions (tests/golden/wilson8.json) agree with the
    independent normal-equation route on every (source, shift), and that route met
    its residual bound: the golden values do not rest on the shifted recurrences alone."""
    import json
    from pathlib import Path
    g = json.loads((Path(__file__).resolve().parent / "golden" / "wilson8.json").read_text())
    assert len(g["sources"]) == 4
    for s in g["sources"]:
        assert s["status"] == "ok"
        assert s["true_res_max"] < 5e-12
        assert s["normal_cg_true_res_max"] < 1e-13
        assert s["normal_cg_max_rel_diff"] < 1e-9
        yn = np.array(s["yn_sample_re"]) + 1j * np.array(s["yn_sample_im"])
        ys = np.array(s["y_sample_re"]) + 1j * np.array(s["y_sample_im"])
        assert np.abs(ys - yn).max() <= 1e-9 * np.abs(yn).max()
