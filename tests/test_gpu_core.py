"""GPU parity of the HIP path against the CPU oracle (small lattices, element by element).

Tolerances:
  * apply_A FP64: relative 1e-14 (a few roundings of ~50-term sums).
  * apply_A FP32: relative 2e-6 (FP32 rounding of inputs, links and sums).
  * shifted CG at a fixed iteration: relative 1e-10. The GPU and the oracle sum
    the dot products in different orders; a Krylov recurrence amplifies those
    rounding differences mildly over tens of iterations.
  * converged solutions: both meet the tolerance 1e-12 on the true residual, so
    they agree to about cond * 1e-12; checked at 1e-9 relative, and the GPU's own
    FP64 true residual at 5e-12.
  * conv_iter: floating point decides it. With the seed at the centre of a nearly
    +-symmetric spectrum CG lowers the residual only every second step, so a
    last-bit difference in the freeze test moves it by 2: identical or within 2.
"""
import numpy as np
import pytest

import synth
from oracle import quadrature as quad
from oracle import solvers, ss, wilson
from tests.helpers import case, to_dev, to_host, vec_err

pytestmark = pytest.mark.gpu

CFG1 = synth.CONFIGS["wilson4_fp64"]


@pytest.fixture(scope="module")
def cfg1():
    U = CFG1.gauge()
    A = wilson.hermitian_wilson(U, CFG1.dims, CFG1.kappa)
    return U, A


def make_ctx(S, dims, kappa, U, link_reals=18):
    c = S.Context(dims, kappa)
    c.set_gauge(U, link_reals)
    return c


@pytest.mark.parametrize("dims,nsrc", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 3), ((6, 4, 5, 3), 2),
                                       ((8, 8, 8, 8), 5), ((3, 5, 7, 2), 1)])
def test_apply_A_fp64(sscg, dims, nsrc):
    case(f"apply_A fp64 dims={dims} nsrc={nsrc}")
    U = synth.gauge_field(dims, 0.5, 11)
    A = wilson.hermitian_wilson(U, dims, 0.13)
    V = int(np.prod(dims))
    x = synth.sources(V, nsrc, 12)
    c = make_ctx(sscg, dims, 0.13, U)
    xd = to_dev(x)
    yd = to_dev(np.zeros_like(x))
    c.apply_A(xd, yd)
    y = to_host(yd).reshape(nsrc, -1)
    ref = np.array([A @ xv for xv in x.reshape(nsrc, -1)])
    assert vec_err(y, ref) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 2, 5), (8, 8, 8, 8), (3, 5, 7, 2)])
@pytest.mark.parametrize("ct,nr,tbs", [(1, 1, 64), (2, 2, 256), (3, 4, 64), (16, 1, 512), (5, 2, 128),
                                       (-1, 1, 0), (-1, 2, 0)])
def test_apply_A_tile_kernel(sscg, monkeypatch, dims, ct, nr, tbs):
    """The tile dslash (tiles of tbs sites marching through ct time slices, a ragged
    last t-range, tiles with faces in y and z or spanning the lattice) and the
    direction-split dslash (ct = -1: one wavefront per direction, 64-site blocks with a
    ragged last block) equal the sparse A in FP64 and the site-parallel kernel in FP64
    and FP32 (18- and 12-real links); where no tile of tbs sites fits the lattice the
    site-parallel kernel runs."""
    case(f"apply_A tile kernel dims={dims} ct={ct} nr={nr} tbs={tbs}")
    U = synth.gauge_field(dims, 0.5, 13)
    A = wilson.hermitian_wilson(U, dims, 0.13)
    V = int(np.prod(dims))
    nsrc = 3
    x = synth.sources(V, nsrc, 14)
    ref = np.array([A @ xv for xv in x.reshape(nsrc, -1)])
    out = {}
    for k in ("plain", "march"):
        monkeypatch.setenv("SSCG_NR", str(nr))
        monkeypatch.setenv("SSCG_TBS", str(tbs))
        monkeypatch.setenv("SSCG_CT", "0" if k == "plain" else str(ct))
        for prec, lr in ((sscg.FP64, 18), (sscg.MIXED, 18), (sscg.MIXED, 12)):
            c = make_ctx(sscg, dims, 0.13, U, lr)
            yd = to_dev(np.zeros_like(x))
            c.apply_A(to_dev(x), yd, prec=prec)
            out[k, prec, lr] = to_host(yd).reshape(nsrc, -1)
            c.close()
    assert vec_err(out["march", sscg.FP64, 18], ref) < 1e-14
    assert vec_err(out["march", sscg.FP64, 18], out["plain", sscg.FP64, 18]) < 1e-15
    for lr in (18, 12):
        assert vec_err(out["march", sscg.MIXED, lr], out["plain", sscg.MIXED, lr]) < 1e-6
        assert vec_err(out["march", sscg.MIXED, lr], ref) < 2e-6


@pytest.mark.parametrize("link_reals", [18, 12])
def test_apply_A_fp32(sscg, cfg1, link_reals):
    case(f"apply_A fp32 link_reals={link_reals}")
    U, A = cfg1
    x = synth.sources(CFG1.V, 2, 3)
    c = make_ctx(sscg, CFG1.dims, CFG1.kappa, U, link_reals)
    yd = to_dev(np.zeros_like(x))
    c.apply_A(to_dev(x), yd, prec=sscg.MIXED)
    y = to_host(yd).reshape(2, -1)
    ref = np.array([A @ xv for xv in x.reshape(2, -1)])
    assert vec_err(y, ref) < 2e-6


def test_shifted_cg_fixed_iteration(sscg, cfg1):
    """Iterates after k = 20 steps equal the oracle's (FOM iterates of every shift)."""
    case("shifted CG fixed k=20")
    U, A = cfg1
    v = CFG1.sources().reshape(CFG1.L, -1)
    z, zeta = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    snap = {}

    def rec(k, st):
        if k == 19:
            snap["X"] = st["X"].copy()

    solvers.shifted_cg(lambda x: A @ x, v[0], z, CFG1.gamma, CFG1.tol, maxiter=20, record=rec)
    c = make_ctx(sscg, CFG1.dims, CFG1.kappa, U)
    y = to_dev(np.zeros((1, CFG1.N, CFG1.n)))
    r = c.shifted_cg_solve(to_dev(v), z, CFG1.gamma, y, sscg.default_opts(maxiter=20, poll_every=7))
    assert r.status == sscg.ENOTCONV
    assert r.iters[0] == 20
    assert vec_err(to_host(y).reshape(CFG1.N, -1), snap["X"]) < 1e-10


def test_shifted_cg_converged(sscg, cfg1):
    case("shifted CG converged cfg1")
    U, A = cfg1
    v = CFG1.sources().reshape(CFG1.L, -1)
    z, zeta = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    ref = solvers.shifted_cg(lambda x: A @ x, v[0], z, CFG1.gamma, CFG1.tol)
    c = make_ctx(sscg, CFG1.dims, CFG1.kappa, U)
    y = to_dev(np.zeros((1, CFG1.N, CFG1.n)))
    r = c.shifted_cg_solve(to_dev(v), z, CFG1.gamma, y)
    assert r.status == sscg.OK
    Y = to_host(y).reshape(CFG1.N, -1)
    assert vec_err(Y, ref.Y) < 1e-9
    assert np.all(np.abs(r.conv_iter[0] - ref.conv_iter) <= 2)
    assert r.true_res.max() < 5e-12
    tr = solvers.true_residuals(lambda x: A @ x, v[0], z, Y)
    assert tr.max() < 5e-12


@pytest.mark.parametrize("L", [1, 2, 7])
def test_free_field_block_ss(sscg, L):
    """Block SS with L sources (Sec. 2.1, block form) on the free field, whose spectrum
    is known in closed form: at 4^4 and kappa = 0.12 the eigenvalues nearest 0 are
    +-0.04, each six-fold, and the next |lambda| is 0.369. The interval [-0.03, 0.03]
    holds no eigenvalue, so nothing may be reported there; [-0.05, 0.05] gives +-0.04
    with multiplicity min(L, 6) (the moments of L sources span at most L vectors of an
    eigenspace), with orthonormal eigenvectors."""
    case(f"free-field block SS L={L}")
    dims, kappa = (4, 4, 4, 4), 0.12
    spec = wilson.free_field_spectrum(dims, kappa)
    assert np.sum(np.abs(spec) <= 0.05) == 12 and np.sum(np.abs(spec) <= 0.03) == 0
    U = synth.unit_gauge(dims)
    c = make_ctx(sscg, dims, kappa, U)
    vd = to_dev(synth.sources(256, L, 3).reshape(L, -1))
    out = c.ss_eigs(sscg.default_ss_params(gamma=0.0, rho=0.03, beta=0.25, N=16, M=8), vd, max_eigs=32)
    assert out.n_found == 0
    out = c.ss_eigs(sscg.default_ss_params(gamma=0.0, rho=0.05, beta=0.25, N=16, M=8), vd, max_eigs=32)
    m = min(L, 6)
    assert out.n_found == 2 * m
    assert np.abs(np.sort(out.lam) - np.array([-0.04] * m + [0.04] * m)).max() < 1e-12
    assert out.res.max() < 1e-8
    X = to_host(out.X).reshape(2 * m, -1)
    assert np.abs(X.conj() @ X.T - np.eye(2 * m)).max() < 1e-8


def test_moments(sscg, cfg1):
    case("ss_moments")
    rng = np.random.default_rng(5)
    L, N, M = 2, 16, 8
    Y = rng.standard_normal((L, N, CFG1.n)) + 1j * rng.standard_normal((L, N, CFG1.n))
    z, zeta = quad.line_nodes(N, 0.0, 0.2, 0.25)
    w = quad.line_weights(zeta)
    ref = ss.moments(Y, zeta, w, M)
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    s = to_dev(np.zeros((L, M, CFG1.n)))
    c.ss_moments(to_dev(Y), N, quad.moment_coefficients(zeta, w, M), s)
    assert vec_err(to_host(s), ref) < 1e-14


def test_ss_eigs_many_columns(sscg, cfg1):
    """Rayleigh-Ritz on 96 moment columns (M = 16, 6 sources) over an interval with 144
    eigenvalues, so the kept basis has more than 64 vectors: the Gram and basis-change
    products run over more than one 64-column tile, with ragged last tiles. Every
    reported pair is certified against the dense spectrum by its residual."""
    case("ss_eigs 96 columns, rank > 64")
    U, A = cfg1
    lo, hi = 0.195, 0.6
    w = CFG1.with_(gamma=0.5 * (lo + hi), rho=0.5 * (hi - lo), L=6, N=32, M=16)
    V = synth.sources(w.V, w.L, w.seed).reshape(w.L, -1)
    c = make_ctx(sscg, w.dims, w.kappa, U)
    p = sscg.default_ss_params(gamma=w.gamma, rho=w.rho, beta=w.beta, N=w.N, M=w.M, rank_tol=1e-7)
    out = c.ss_eigs(p, to_dev(V), max_eigs=96)
    assert out.info.rank > 64  # (the oracle's Rayleigh-Ritz keeps 91 directions here)
    assert out.n_found >= 1 and out.res.max() <= 1e-6
    ev = np.linalg.eigvalsh(A.toarray())
    X = to_host(out.X).reshape(len(out.lam), -1)
    for lam, x, r in zip(out.lam, X, out.res):
        assert lo <= lam <= hi
        assert np.min(np.abs(ev - lam)) <= r + 1e-13
        assert abs(np.linalg.norm(x) - 1) < 1e-12
        assert abs(np.linalg.norm(A @ x - lam * x) - r) <= 1e-3 * r + 1e-13


@pytest.mark.parametrize("method", ["rr", "hankel"])
def test_ss_eigs_window(sscg, cfg1, method):
    """Interval [0.195, 0.255] holds the six lowest positive eigenvalues of the 4^4 field."""
    case(f"ss_eigs window {method}")
    U, A = cfg1
    w = CFG1.with_(gamma=0.225, rho=0.03, L=2)
    V = synth.sources(w.V, w.L, w.seed).reshape(w.L, -1)
    ref = ss.ss_eigs(A, V, w.gamma, w.rho, w.beta, w.N, w.M, method=method, rank_tol=1e-7)
    c = make_ctx(sscg, w.dims, w.kappa, U)
    p = sscg.default_ss_params(gamma=w.gamma, rho=w.rho, beta=w.beta, N=w.N, M=w.M,
                               method=sscg.RR if method == "rr" else sscg.HANKEL, rank_tol=1e-7)
    out = c.ss_eigs(p, to_dev(V), max_eigs=16)
    ev = np.linalg.eigvalsh(A.toarray())
    truth = ev[(ev >= w.gamma - w.rho) & (ev <= w.gamma + w.rho)]
    assert out.n_found == len(ref["lam"]) == len(truth) == 6
    # parity with the oracle's own extraction (same method)
    assert np.all(np.abs(out.lam - ref["lam"].real) <= 1e-10 * np.maximum(np.abs(ref["lam"].real), 0.1 * w.rho))
    # every reported pair is certified by its residual (Hermitian A)
    assert np.all(np.abs(out.lam - truth) <= out.res + 1e-13)
    if method == "rr":
        # Rayleigh-Ritz reaches the exact spectrum here; Hankel is limited by its residual
        assert np.all(np.abs(out.lam - truth) <= 1e-10 * np.maximum(np.abs(truth), 0.1 * w.rho))
        assert out.res.max() < 1e-8
    X = to_host(out.X).reshape(len(out.lam), -1)
    for lam, x, r in zip(out.lam, X, out.res):
        assert abs(np.linalg.norm(x) - 1) < 1e-12
        assert np.linalg.norm(A @ x - lam * x) < max(2 * r, 1e-12)
