"""GPU parity at the full workload sizes, in the launch configuration the benchmark uses.

8^4 FP64 (32 shifts, 4 sources): every entry of every solution against the
oracle's shifted CG run in the test, the stored entries against the independent
normal-equation solutions (tests/golden/wilson8.json, written by
tests/golden/make_golden.py), per-shift convergence iterations (within 2: CG with a
centred seed lowers the residual every second step), residuals from the oracle's
matrix below 5e-12, and an empty eigen-interval as the reference spectrum predicts. A window at the low end
of the 8^4 spectrum checks eigenvalues against the reference spectrum (1e-10
relative) with residuals below 1e-8.

Larger lattices: at 16^3 x 32 every solution of all 8 sources is certified with the
oracle's explicit matrix; at 24^3 x 48 (all 8 sources, FP64 and both mixed modes)
and for the batched 8^4/12^4/16^4 workload, properties that hold at any size are
checked with the oracle's row-wise matrix on sampled sites: sampled entries of
v - (z_j - A) y_j, sampled rows of A x - lambda x against the reported residual,
and the batched run against the per-problem runs.
"""
import json
from pathlib import Path

import numpy as np
import pytest

import synth
from oracle import quadrature as quad
from oracle import solvers, wilson
from tests.helpers import case, to_dev, to_host, vec_err

pytestmark = pytest.mark.gpu
GOLD = Path(__file__).resolve().parent / "golden" / "wilson8.json"


@pytest.fixture(scope="module")
def gold():
    return json.loads(GOLD.read_text())


@pytest.fixture(scope="module")
def w8(sscg):
    w = synth.CONFIGS["wilson8_fp64"]
    U = w.gauge()
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U)
    return w, U, c


@pytest.fixture(scope="module")
def w8_oracle(w8):
    """The oracle's explicit A and its shifted CG for every source of the 8^4 workload."""
    w, U, c = w8
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)
    V = w.sources().reshape(w.L, -1)
    z, _ = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    runs = [solvers.shifted_cg(lambda x: A @ x, V[l], z, w.gamma, w.tol) for l in range(w.L)]
    return A, V, z, runs


def test_wilson8_shifted_cg_every_entry(sscg, w8, w8_oracle, gold):
    """All 128 solutions (4 sources x 32 shifts) of the 8^4 FP64 solve, entry by entry:
    against the oracle's shifted CG run on the same inputs (per shift, max_i |dy_i| at
    most 1e-9 max_i |y_i|: the two sum their dot products in different orders, and
    shifts that stop an iteration apart differ by about the tolerance times the
    condition number); at the 16 stored indices against the normal-equation solutions
    of the golden file (an independent route, see make_golden.py); and with residuals
    ||v - (z_j I - A) y_j|| / ||v|| below 5e-12 computed from the oracle's matrix, not
    from the library's own true residual."""
    case("8^4 FP64 shifted CG, every entry vs oracle")
    w, U, c = w8
    A, V, z, runs = w8_oracle
    y = to_dev(np.zeros((w.L, w.N, w.n)))
    r = c.shifted_cg_solve(to_dev(V), z, w.gamma, y)
    assert r.status == sscg.OK
    Y = to_host(y)
    del y
    idx = np.array(gold["sample_index"])
    for l, g in enumerate(gold["sources"]):
        ref = runs[l]
        assert abs(int(r.iters[l]) - ref.iters) <= 2 and abs(int(r.iters[l]) - g["iters"]) <= 2
        assert np.all(np.abs(r.conv_iter[l] - ref.conv_iter) <= 2)
        assert np.all(np.abs(r.conv_iter[l] - np.array(g["conv_iter"])) <= 2)
        assert vec_err(Y[l], ref.Y) <= 1e-9
        yn = np.array(g["yn_sample_re"]) + 1j * np.array(g["yn_sample_im"])
        assert vec_err(Y[l][:, idx], yn) <= 1e-9
        AY = (A @ Y[l].T).T
        res = np.linalg.norm(V[l][None, :] - (z[:, None] * Y[l] - AY), axis=1) / np.linalg.norm(V[l])
        assert res.max() < 5e-12


def test_wilson8_specified_interval_is_empty(sscg, w8, gold):
    case("8^4 ss_eigs specified interval")
    w, U, c = w8
    lam_ref = np.array(gold["lowest_eigs"]["lam"])
    assert np.all(np.abs(lam_ref) > w.rho)   # no eigenvalue in [-0.1, 0.1]
    p = sscg.default_ss_params(gamma=w.gamma, rho=w.rho, beta=w.beta, N=w.N, M=w.M)
    out = c.ss_eigs(p, to_dev(w.sources().reshape(w.L, -1)), max_eigs=64)
    assert out.n_found == 0


@pytest.mark.parametrize("lo,hi,beta,M", [(0.3700, 0.3735, 0.5, 8), (0.3740, 0.3760, 0.5, 8)])
def test_wilson8_window_eigenpairs(sscg, w8, gold, lo, hi, beta, M):
    case(f"8^4 eigen window [{lo}, {hi}] beta={beta}")
    w, U, c = w8
    lam_ref = np.array(gold["lowest_eigs"]["lam"])
    truth = np.sort(lam_ref[(lam_ref >= lo) & (lam_ref <= hi)])
    assert len(truth) >= 2
    gamma, rho = 0.5 * (lo + hi), 0.5 * (hi - lo)
    p = sscg.default_ss_params(gamma=gamma, rho=rho, beta=beta, N=32, M=M)
    out = c.ss_eigs(p, to_dev(w.sources().reshape(w.L, -1)), max_eigs=32)
    assert out.n_found == len(truth)
    assert np.all(np.abs(out.lam - truth) <= 1e-10 * np.abs(truth))
    assert out.res.max() < 1e-8
    # sampled rows of A x - lambda x from the oracle agree with the reported residual
    X = to_host(out.X)
    sites = np.random.default_rng(3).choice(w.V, 32, replace=False)
    for k in range(len(out.lam)):
        rows = wilson.apply_rows(U, w.dims, w.kappa, X[k], sites)
        r = rows - out.lam[k] * X[k].reshape(-1, 12)[sites]
        assert np.abs(r).max() <= out.res[k] + 1e-13


def sampled_shift_residuals(U, dims, kappa, v, z, y, sites):
    """max over shifts of max_i |(v - (z_j - A) y_j)_i| on the rows of the sampled sites."""
    worst = 0.0
    for j, zj in enumerate(z):
        Ay = wilson.apply_rows(U, dims, kappa, y[j], sites)
        r = v.reshape(-1, 12)[sites] - (zj * y[j].reshape(-1, 12)[sites] - Ay)
        worst = max(worst, np.abs(r).max())
    return worst


def test_wilson16x32_mixed_all_sources(sscg):
    """The 16^3 x 32 workload in its specified recipe (SSCG_MIXED: FP32 dslash, seed and
    shift vectors after the switch, FP64 reliable updates every 50 iterations), all 8
    sources x 32 nodes: every one of the 256 solutions is certified with the oracle's
    explicit matrix, ||v - (z_j I - A) y_j|| / ||v|| <= 1e-10 (100 times the
    tolerance, the bound the library's own FP64 check applies), and those residuals
    agree with the ones the library reports."""
    w = synth.CONFIGS["wilson16x32_mixed"]
    case(f"{w.name} SSCG_MIXED, all {w.L} sources, oracle residuals")
    U = w.gauge()
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U, w.link_reals)
    V = w.sources().reshape(w.L, -1)
    z, _ = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    y = to_dev(np.zeros((w.L, w.N, w.n)))
    r = c.shifted_cg_solve(to_dev(V), z, w.gamma, y,
                           sscg.default_opts(prec=sscg.MIXED, ru_interval=w.ru_interval, switch_tol=w.switch_tol))
    assert r.status == sscg.OK
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)
    for l in range(w.L):
        Y = to_host(y[l])
        res = np.linalg.norm(V[l][None, :] - (z[:, None] * Y - (A @ Y.T).T), axis=1) / np.linalg.norm(V[l])
        assert res.max() <= 1e-10, (l, res.max())
        assert np.abs(res - r.true_res[l]).max() <= 1e-3 * res.max() + 1e-15
    del y
    c.close()


@pytest.mark.parametrize("lo,hi,mode,method", [(0.3650, 0.3661, "fp64", "rr"), (0.3650, 0.3661, "mixed_shifts", "rr"),
                                                (0.3650, 0.3661, "fp64", "hankel"), (-0.3661, -0.3655, "fp64", "rr"),
                                                (-0.3661, -0.3655, "mixed_shifts", "rr")])
def test_wilson16x32_window_eigenpairs(sscg, lo, hi, mode, method):
    """Windows of the 16^3 x 32 field that hold eigenvalues (the reference spectrum,
    tests/golden/spectrum_wilson16x32_mixed.json, written by the oracle, covers every
    |lambda| <= 0.36686, so it is complete inside them): the lowest positive and the
    highest negative eigenvalue, each at least 1.3 rho from its nearest neighbour. Each
    is found within 1e-10 max(|lambda|, 0.1 rho) of the reference with ||A x - lambda x||
    below 1e-8, in FP64 and with FP32 shift vectors, by Rayleigh-Ritz and block Hankel;
    sampled rows of A x - lambda x from the oracle's row-wise matrix bound the reported
    residual."""
    w = synth.CONFIGS["wilson16x32_mixed"]
    case(f"16^3x32 eigen window [{lo}, {hi}] {mode} {method}")
    ref = json.loads((GOLD.parent / "spectrum_wilson16x32_mixed.json").read_text())
    lam_ref = np.array(ref["lam"])
    assert np.max(np.abs(lam_ref)) > max(abs(lo), abs(hi))
    truth = np.sort(lam_ref[(lam_ref >= lo) & (lam_ref <= hi)])
    assert len(truth) == 1
    U = w.gauge()
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U, w.link_reals)
    prec = sscg.FP64 if mode == "fp64" else sscg.MIXED_SHIFTS
    gamma, rho = 0.5 * (lo + hi), 0.5 * (hi - lo)
    p = sscg.default_ss_params(gamma=gamma, rho=rho, beta=0.5, N=32, M=8,
                               method=sscg.RR if method == "rr" else sscg.HANKEL,
                               solve=sscg.default_opts(prec=prec, ru_interval=w.ru_interval, switch_tol=w.switch_tol))
    V = w.sources().reshape(w.L, -1)[:4]
    out = c.ss_eigs(p, to_dev(V), max_eigs=16)
    assert out.status == sscg.OK
    assert out.n_found == len(truth)
    assert np.all(np.abs(out.lam - truth) <= 1e-10 * np.maximum(np.abs(truth), 0.1 * rho))
    assert out.res.max() < 1e-8
    X = to_host(out.X)
    sites = np.random.default_rng(11).choice(w.V, 16, replace=False)
    for k in range(len(out.lam)):
        rows = wilson.apply_rows(U, w.dims, w.kappa, X[k], sites)
        r = rows - out.lam[k] * X[k].reshape(-1, 12)[sites]
        assert np.abs(r).max() <= out.res[k] + 1e-13
    c.close()


def test_batched_workload_equals_single_runs(sscg):
    names = synth.BATCH
    case("batched 8^4 / 12^4 / 16^4 mixed")
    ctxs, vs, zs, ys, Us, Vs = [], [], [], [], [], []
    opts = sscg.default_opts(prec=sscg.MIXED, ru_interval=50, switch_tol=1e-6)
    for nm in names:
        w = synth.CONFIGS[nm]
        U = w.gauge()
        c = sscg.Context(w.dims, w.kappa)
        c.set_gauge(U)
        V = w.sources().reshape(w.L, -1)
        z, _ = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
        ctxs.append(c)
        vs.append(to_dev(V))
        zs.append(z)
        ys.append(to_dev(np.zeros((w.L, w.N, w.n))))
        Us.append(U)
        Vs.append(V)
    res = sscg.batch_solve(ctxs, vs, zs, [synth.CONFIGS[nm].gamma for nm in names], ys, opts)
    for i, nm in enumerate(names):
        w = synth.CONFIGS[nm]
        assert res[i].status == sscg.OK, nm
        assert res[i].true_res.max() < 1e-10, nm
        y1 = to_dev(np.zeros((w.L, w.N, w.n)))
        r1 = ctxs[i].shifted_cg_solve(vs[i], zs[i], w.gamma, y1, opts)
        assert r1.status == sscg.OK
        # the mixed switch happens at a poll boundary common to the whole batch, so a
        # member's run alone may switch earlier; both meet the same residual bound
        assert vec_err(to_host(ys[i]), to_host(y1)) < 1e-8, nm
        sites = np.random.default_rng(5 + i).choice(w.V, 6, replace=False)
        worst = sampled_shift_residuals(Us[i], w.dims, w.kappa, Vs[i][0], zs[i], to_host(ys[i])[0], sites)
        assert worst <= 2e-10 * np.linalg.norm(Vs[i][0]), nm


def test_batched_fp64_is_bitwise_the_single_runs(sscg, monkeypatch):
    """With one fixed launch shape, each problem of an FP64 batch (two lattices of
    different size, own intervals and shift counts) gives exactly the bits of its run
    alone: the grouped launches share kernels and reductions do not depend on the
    batch."""
    case("batched FP64 bitwise vs single")
    for k, v in dict(SSCG_NR="2", SSCG_BS="128", SSCG_WBATCH="4", SSCG_UNROLL="2", SSCG_XCD="1",
                     SSCG_CT="0").items():
        monkeypatch.setenv(k, v)
    probs = []
    for dims, kappa, seed, (gamma, rho), N in (((4, 4, 4, 4), 0.12, 31, (0.0, 0.2), 16),
                                               ((6, 4, 4, 6), 0.125, 32, (0.05, 0.1), 12)):
        U = synth.gauge_field(dims, 0.5, seed)
        V = synth.sources(int(np.prod(dims)), 2, seed).reshape(2, -1)
        z, _ = quad.line_nodes(N, gamma, rho, 0.25)
        c = sscg.Context(dims, kappa)
        c.set_gauge(U)
        probs.append((c, V, z, gamma))
    opts = sscg.default_opts()
    ys = [to_dev(np.zeros((2, len(z), V.shape[1]))) for c, V, z, g in probs]
    res = sscg.batch_solve([p[0] for p in probs], [to_dev(p[1]) for p in probs], [p[2] for p in probs],
                           [p[3] for p in probs], ys, opts)
    for (c, V, z, g), yb, rb in zip(probs, ys, res):
        y1 = to_dev(np.zeros((2, len(z), V.shape[1])))
        r1 = c.shifted_cg_solve(to_dev(V), z, g, y1, opts)
        assert rb.status == r1.status == sscg.OK
        assert np.array_equal(to_host(yb), to_host(y1))
        assert np.array_equal(rb.conv_iter, r1.conv_iter)


@pytest.fixture(scope="module")
def w24(sscg):
    w = synth.CONFIGS["wilson24x48"]
    return w, w.gauge()


@pytest.mark.parametrize("prec,link_reals,bound", [("fp32", 12, 2e-6), ("fp64", 18, 1e-13)])
def test_wilson24x48_dslash_sampled_rows(sscg, w24, prec, link_reals, bound):
    """The dslash at the large workload's full size (24^3 x 48, 8 sources), in the
    launch shape the autotuner picks for apply_A (as the benchmark times it): sampled
    rows of A x against the oracle's row-wise matrix."""
    w, U = w24
    case(f"24^3x48 apply_A {prec} links={link_reals}")
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U, link_reals)
    X = w.sources().reshape(w.L, -1)
    xd = to_dev(X)
    yd = to_dev(np.zeros_like(X))
    c.apply_A(xd, yd, prec=sscg.MIXED if prec == "fp32" else sscg.FP64)
    Y = to_host(yd)
    sites = np.random.default_rng(6).choice(w.V, 24, replace=False)
    for l in (0, 5, 7):
        rows = wilson.apply_rows(U, w.dims, w.kappa, X[l], sites)
        got = Y[l].reshape(-1, 12)[sites]
        assert np.abs(got - rows).max() <= bound * np.abs(rows).max()
    c.close()


def test_wilson24x48_window_eigenpair(sscg, w24):
    """A window of the 24^3 x 48 field that holds an eigenvalue, [0.3450, 0.3457],
    around the field's smallest |lambda| (two sources, N = 32, M = 8, beta = 0.5,
    moments summed inside the solve). The reference spectrum
    (tests/golden/spectrum_wilson24x48.json, the six smallest |lambda| from the
    oracle's Lanczos on A^2) holds every |lambda| below its fifth value, 0.34621, so
    it is complete inside this window and its mirror: one eigenvalue, 0.3454945964,
    and none in [-0.3457, -0.3450]. The pair matches it to 1e-10 in FP64 and with FP32
    shift vectors, and is certified by the oracle's explicit matrix: ||A x - lambda x||
    / ||x|| below 1e-8 and at most 1.5 times the reported residual."""
    import torch
    w, U = w24
    case("24^3x48 eigen window [0.3450, 0.3457]")
    lo, hi = 0.3450, 0.3457
    ref = np.array(json.loads((GOLD.parent / "spectrum_wilson24x48.json").read_text())["lam"])
    assert np.sort(np.abs(ref))[4] > hi
    truth = ref[(ref >= lo) & (ref <= hi)]
    assert len(truth) == 1 and not np.any((ref >= -hi) & (ref <= -lo))
    gamma, rho = 0.5 * (lo + hi), 0.5 * (hi - lo)
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U, 18)
    V = to_dev(w.sources().reshape(w.L, -1)[:2])
    found = {}
    for mode in ("fp64", "mixed_shifts"):
        prec = sscg.FP64 if mode == "fp64" else sscg.MIXED_SHIFTS
        p = sscg.default_ss_params(gamma=gamma, rho=rho, beta=0.5, N=32, M=8, moments_in_loop=1,
                                   solve=sscg.default_opts(prec=prec, ru_interval=w.ru_interval,
                                                           switch_tol=w.switch_tol))
        out = c.ss_eigs(p, V, max_eigs=8)
        assert out.status == sscg.OK
        assert out.n_found == 1
        assert out.res.max() < 1e-8
        found[mode] = (float(out.lam[0]), float(out.res[0]), to_host(out.X)[0].reshape(-1))
        print(f"[case] {mode}: lambda {out.lam[0]:.12f} res {out.res[0]:.2e} seed iterations {out.info.iters}",
              flush=True)
    l64, l32 = found["fp64"][0], found["mixed_shifts"][0]
    assert abs(l64 - l32) <= 1e-10 * abs(l64)
    assert abs(l64 - truth[0]) <= 1e-10 * abs(truth[0])
    p = sscg.default_ss_params(gamma=-gamma, rho=rho, beta=0.5, N=32, M=8, moments_in_loop=1)
    assert c.ss_eigs(p, V, max_eigs=8).n_found == 0
    del V
    torch.cuda.empty_cache()
    c.close()
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)  # the explicit matrix (about a minute)
    for mode, (lam, res, x) in found.items():
        x = x / np.linalg.norm(x)
        r = np.linalg.norm(A @ x - lam * x)
        assert r < 1e-8
        assert r <= 1.5 * res + 1e-13
        print(f"[case] {mode}: oracle residual {r:.2e}", flush=True)


def sampled_rows_residual(U, dims, kappa, v, z, y_dev, sites):
    """max over (node, sampled site) of |(v - (z_j I - A) y_j)_i| / ||v|| with the
    oracle's row-wise operator: only the entries of y_j at the sampled sites and their
    eight neighbours are copied to the host (the full solutions of the large lattice
    do not fit there), placed in a zero vector of full length for apply_rows."""
    import torch
    Vn = int(np.prod(dims))
    cs = wilson.coords(dims)[sites]
    need = [sites]
    for mu in range(4):
        for step in (1, -1):
            cc = cs.copy()
            cc[:, mu] = (cc[:, mu] + step) % dims[mu]
            need.append(wilson.site_index(cc, dims))
    need = np.unique(np.concatenate(need))
    idx = torch.from_numpy(need).to(y_dev.device)
    sub = y_dev.view(len(z), Vn, 12).index_select(1, idx).cpu().numpy()   # [N][len(need)][12]
    vs = v.reshape(-1, 12)[sites]
    worst = 0.0
    full = np.zeros((Vn, 12), dtype=np.complex128)
    for j, zj in enumerate(z):
        full[need] = sub[j]
        Ay = wilson.apply_rows(U, dims, kappa, full, sites)
        r = vs - (zj * full[sites] - Ay)
        worst = max(worst, float(np.abs(r).max()))
    return worst / np.linalg.norm(v)


@pytest.mark.parametrize("mode", ["fp64", "mixed12", "mixed_shifts"])
def test_wilson24x48_solve_all_sources(sscg, w24, mode):
    """The large workload (24^3 x 48, 64 nodes on lines around [-0.05, 0.05] with
    beta = 0.4, all 8 sources) in FP64 and with FP32 shift vectors (SSCG_MIXED_SHIFTS):
    the library's FP64 true residual of each of the 512 solutions below 1e-10 (5e-11
    in FP64), and sampled rows of v - (z_j I - A) y_j below 1e-10 ||v|| for every
    node of sources 0 and 7 with the oracle's row-wise operator. In the specified
    recipe (SSCG_MIXED: FP32 spinors with 12-real links after the switch, FP64
    reliable updates) the result must state its error truthfully."""
    import torch
    w, U = w24
    case(f"24^3x48 {mode} solve, all {w.L} sources")
    prec = {"fp64": sscg.FP64, "mixed12": sscg.MIXED, "mixed_shifts": sscg.MIXED_SHIFTS}[mode]
    c = sscg.Context(w.dims, w.kappa)
    c.set_gauge(U, 12 if mode == "mixed12" else 18)
    V = w.sources().reshape(w.L, -1)
    z, _ = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    y = torch.zeros((w.L, w.N, w.n), dtype=torch.complex128, device="cuda:0")
    r = c.shifted_cg_solve(to_dev(V), z, w.gamma, y,
                           sscg.default_opts(prec=prec, ru_interval=w.ru_interval, switch_tol=w.switch_tol))
    sites = np.random.default_rng(7).choice(w.V, 4, replace=False)
    if mode == "mixed12":
        # the FP32 seed of SSCG_MIXED loses the FP64 convergence of this indefinite seed
        # on some sources (many more iterations); what must hold is that the result
        # states its error: the status follows the FP64 true residuals (100 tol), and
        # those bound the oracle's sampled residual rows
        assert r.status in (sscg.OK, sscg.EINACCURATE)
        assert (r.status == sscg.EINACCURATE) == bool(r.true_res.max() > 100 * w.tol)
        for l in (0, 7):
            worst = sampled_rows_residual(U, w.dims, w.kappa, V[l], z, y[l], sites)
            assert worst <= r.true_res[l].max() * 1.001 + 1e-14
    else:
        assert r.status == sscg.OK
        assert r.true_res.max() < (5e-11 if mode == "fp64" else 1e-10)
        for l in (0, 7):
            assert sampled_rows_residual(U, w.dims, w.kappa, V[l], z, y[l], sites) <= 1e-10
    print(f"[case] {mode}: seed iterations {r.iters.tolist()}, max true residual {r.true_res.max():.2e}", flush=True)
    del y
    torch.cuda.empty_cache()
    c.close()
