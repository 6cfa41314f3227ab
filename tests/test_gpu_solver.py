"""GPU shifted-CG behaviour: determinism, launch shapes, mixed precision, batching,
several sources, and the failure paths forced from the host.

Bars:
  * results must not depend on how often the host polls or on graph replay:
    bitwise equal. Every reduction is two-stage with partials of a fixed
    granularity (64 sites for the dslash, 512 entries for the vector kernels)
    summed in a fixed order, also independent of the launch shapes;
  * across launch shapes (block size, sources per thread, shift batch, unrolling,
    XCD order) different kernel instantiations may contract multiply-adds
    differently; the Krylov recurrence amplifies such last-bit differences over a
    few hundred iterations, so the bar is 1e-11 relative (100 times below the
    oracle parity bar) and convergence iterations within 2;
  * mixed precision: every shift's FP64 true residual <= 1e-10 (tolerance 1e-12
    on the implicit residual, FP32 arithmetic after the switch at 1e-6; the
    residual gap is bounded by ~eps_32 * switch_tol * cond) and the solution
    within 1e-9 of the FP64 oracle's;
  * a batched FP64 solve equals the single-problem solves of its members to the
    same 1e-11 (the batch may be tuned to other launch shapes).
"""
import numpy as np
import pytest

import synth
from oracle import quadrature as quad
from oracle import solvers, wilson
from tests.helpers import case, to_dev, to_host, vec_err

pytestmark = pytest.mark.gpu

CFG1 = synth.CONFIGS["wilson4_fp64"]


@pytest.fixture(scope="module")
def prob():
    U = CFG1.gauge()
    A = wilson.hermitian_wilson(U, CFG1.dims, CFG1.kappa)
    V = synth.sources(CFG1.V, 3, 21).reshape(3, -1)
    z, _ = quad.line_nodes(CFG1.N, CFG1.gamma, CFG1.rho, CFG1.beta)
    return U, A, V, z


def solve(S, U, V, z, sigma=0.0, dims=CFG1.dims, kappa=CFG1.kappa, link_reals=18, **opts):
    c = S.Context(dims, kappa)
    c.set_gauge(U, link_reals)
    L = V.shape[0]
    y = to_dev(np.zeros((L, len(z), V.shape[1])))
    r = c.shifted_cg_solve(to_dev(V), z, sigma, y, S.default_opts(**opts))
    return to_host(y), r


def test_poll_and_graph_do_not_change_results(sscg, prob):
    case("determinism poll/graph")
    U, A, V, z = prob
    y0, r0 = solve(sscg, U, V, z, poll_every=50, use_graph=1)
    y1, r1 = solve(sscg, U, V, z, poll_every=7, use_graph=0)
    y2, r2 = solve(sscg, U, V, z, poll_every=1000, use_graph=1)
    assert np.array_equal(y0, y1) and np.array_equal(y0, y2)
    assert np.array_equal(r0.conv_iter, r1.conv_iter) and np.array_equal(r0.iters, r2.iters)


def test_graphs_kept_across_solves(sscg, prob, monkeypatch):
    """A context keeps its solve-loop graphs between solves and replays them when the
    launch plan is the same; solves of other shifts, source counts and options on one
    context give bitwise what fresh contexts give (fixed launch shapes, so that every
    context runs the same kernels)."""
    case("graph reuse across solves")
    monkeypatch.setenv("SSCG_AUTOTUNE", "0")
    U, A, V, z = prob
    z2 = z * 0.5 + 0.01
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    c.set_gauge(U, 18)
    runs = [(V, z, {}), (V, z2, {}), (V, z, {}), (V[:1], z, {}), (V, z, dict(poll_every=30)),
            (V, z, dict(prec=sscg.MIXED_SHIFTS)), (V, z, {})]
    for Vk, zk, kw in runs:
        y = to_dev(np.zeros((Vk.shape[0], len(zk), Vk.shape[1])))
        r = c.shifted_cg_solve(to_dev(Vk), zk, 0.0, y, sscg.default_opts(**kw))
        y_ref, r_ref = solve(sscg, U, Vk, zk, **kw)
        assert np.array_equal(to_host(y), y_ref), kw
        assert np.array_equal(r.conv_iter, r_ref.conv_iter) and np.array_equal(r.iters, r_ref.iters)
    c.close()


def test_profiling_levels(sscg, prob):
    """Level 1 times every launch (direct launches); level 5 keeps graph replay and
    times every stage of every 5th iteration. Neither changes the results (bitwise),
    the sampled launch averages agree with the full ones, and the launch counts the
    context reports scale the sample to the whole solve. Launches after the last
    source finished (up to the next poll) exit at once: they are neither counted nor
    timed."""
    case("profiling levels")
    U, A, V, z = prob
    y_ref, r_ref = solve(sscg, U, V, z, poll_every=50, use_graph=1)
    out = {}
    for level, graph in ((1, 1), (5, 1), (5, 0)):
        c = sscg.Context(CFG1.dims, CFG1.kappa)
        c.set_gauge(U, 18)
        c.set_profiling(level)
        y = to_dev(np.zeros((V.shape[0], len(z), V.shape[1])))
        r = c.shifted_cg_solve(to_dev(V), z, 0.0, y, sscg.default_opts(poll_every=50, use_graph=graph))
        ms, calls = c.stage_times()
        launches = c.stage_launches()
        assert np.array_equal(to_host(y), y_ref) and np.array_equal(r.iters, r_ref.iters)
        out[level, graph] = (np.array(ms), np.array(calls))
        out["launches", level, graph] = launches
        c.close()
    (ms1, calls1), (ms5, calls5) = out[1, 1], out[5, 1]
    # sampling with direct launches takes the same samples as inside the graphs
    assert np.array_equal(out[5, 0][1][:6], calls5[:6])
    kwork = int(np.max(r_ref.iters))           # iterations in which the source iterated
    launched = int(out["launches", 1, 1][6])   # iterations launched (polls every 50)
    assert launched >= kwork and launched % 50 == 0
    assert calls1[0] == calls1[2] == calls1[4] == kwork and calls1[3] == 0 and np.all(ms1[[0, 2, 4]] > 0)
    # every stage of iterations 2, 7, 12, ... of each 50-iteration poll interval before
    # kwork (the step length is fused into the residual update on this lattice: no
    # alpha stage)
    nsamp = sum(1 for k0 in range(0, launched, 50) for it in range(2, 50, 5) if k0 + it < kwork)
    assert calls5[0] == calls5[2] == calls5[4] == nsamp and np.all(calls5[[1, 3, 5]] == 0)
    # launch counts: one dslash, residual update and shift update per iteration with work
    for key in (("launches", 1, 1), ("launches", 5, 1), ("launches", 5, 0)):
        n = out[key]
        assert n[0] == n[2] == n[4] == kwork and n[6] == launched and n[1] == n[3] == n[5] == 0
    for s in (0, 2, 4):
        a1, a5 = ms1[s] / calls1[s], ms5[s] / calls5[s]
        assert 0.3 < a5 / a1 < 3.0, (s, a1, a5)
    with pytest.raises(sscg.SSCGError):
        c = sscg.Context(CFG1.dims, CFG1.kappa)
        try:
            c.set_profiling(-1)
        finally:
            c.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fused_step_length_is_bitwise_the_same(sscg, prob, monkeypatch, prec):
    """The seed step length formed inside the residual update (small lattices) equals
    the separate alpha kernel's bit for bit: same partials, same summation order. The
    mixed case includes reliable-update iterations."""
    case(f"fused alpha {prec}")
    U, A, V, z = prob
    kw = dict(prec=sscg.MIXED, ru_interval=20, switch_tol=1e-6) if prec == "mixed" else {}
    monkeypatch.setenv("SSCG_NR", "2")           # one fixed launch shape for every run
    out = []
    for fa in ("0", "1"):
        monkeypatch.setenv("SSCG_FUSE_ALPHA", fa)
        out.append(solve(sscg, U, V, z, **kw))
    (y0, r0) = out[0]
    for y1, r1 in out[1:]:
        assert r1.status == r0.status == sscg.OK
        assert np.array_equal(y0, y1)
        assert np.array_equal(r0.conv_iter, r1.conv_iter) and np.array_equal(r0.iters, r1.iters)


@pytest.mark.parametrize("env", [dict(SSCG_NR="1", SSCG_BS="64", SSCG_WBATCH="3", SSCG_XCD="0", SSCG_UNROLL="1"),
                                 dict(SSCG_NR="4", SSCG_BS="128", SSCG_WBATCH="16", SSCG_XCD="1", SSCG_UNROLL="4",
                                      SSCG_NT="1"),
                                 dict(SSCG_NR="2", SSCG_BS="256", SSCG_WBATCH="1", SSCG_XCD="1", SSCG_UNROLL="2"),
                                 dict(SSCG_NR="2", SSCG_TBS="64", SSCG_CT="3", SSCG_XCD="1"),
                                 dict(SSCG_NR="1", SSCG_TBS="64", SSCG_CT="1", SSCG_XCD="0", SSCG_DORDER="2"),
                                 dict(SSCG_NR="2", SSCG_CT="-1", SSCG_XCD="1"),
                                 dict(SSCG_WBATCH="4", SSCG_UNROLL="2", SSCG_BORDER="1", SSCG_NT="1")])
def test_launch_shapes_agree(sscg, prob, monkeypatch, env):
    case(f"launch shapes {env}")
    U, A, V, z = prob
    y_ref, r_ref = solve(sscg, U, V, z)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    y, r = solve(sscg, U, V, z)
    assert vec_err(y, y_ref) < 1e-11
    assert np.all(np.abs(r.conv_iter - r_ref.conv_iter) <= 2)


def test_several_sources_and_seed_shift(sscg, prob):
    case("3 sources, seed 0.07")
    U, A, V, z = prob
    y, r = solve(sscg, U, V, z, sigma=0.07)
    assert r.status == sscg.OK
    for l in range(3):
        ref = solvers.shifted_cg(lambda x: A @ x, V[l], z, 0.07, 1e-12)
        assert vec_err(y[l], ref.Y) < 1e-9
        assert np.all(np.abs(r.conv_iter[l] - ref.conv_iter) <= 2)
        assert r.iters[l] == pytest.approx(ref.iters, abs=2)
    assert r.true_res.max() < 5e-12


@pytest.mark.parametrize("mode,link_reals", [("mixed", 18), ("mixed", 12), ("mixed_shifts", 18)])
def test_mixed_precision_accuracy(sscg, prob, mode, link_reals):
    case(f"{mode} precision link_reals={link_reals}")
    U, A, V, z = prob
    y64, r64 = solve(sscg, U, V, z)
    prec = sscg.MIXED if mode == "mixed" else sscg.MIXED_SHIFTS
    y, r = solve(sscg, U, V, z, prec=prec, ru_interval=20, switch_tol=1e-6, link_reals=link_reals)
    assert r.status == sscg.OK
    assert r.true_res.max() < 1e-10
    for l in range(3):
        tr = solvers.true_residuals(lambda x: A @ x, V[l], z, y[l])
        assert tr.max() < 1e-10
    assert vec_err(y, y64) < 1e-9


def test_mixed_shifts_matches_fp32_emulation(sscg, prob):
    """The FP32-shift mode against the oracle's emulation of the same precision
    schedule (complex64 shift vectors after the switch at 1e-6, FP64 seed): both land
    within 1e-10 of the dense spectral solution and within 1e-10 of each other."""
    case("mixed_shifts vs oracle FP32 emulation")
    U, A, V, z = prob
    lam, W = np.linalg.eigh(A.toarray())
    y, r = solve(sscg, U, V, z, prec=sscg.MIXED_SHIFTS, ru_interval=20, switch_tol=1e-6)
    assert r.status == sscg.OK
    for l in range(V.shape[0]):
        emu = solvers.shifted_cg(lambda x: A @ x, V[l], z, 0.0, 1e-12, fp32_switch=1e-6, fold_every=20)
        c = W.conj().T @ V[l]
        exact = np.array([W @ (c / (zj - lam)) for zj in z])
        for Y in (y[l], emu.Y):
            err = np.linalg.norm(Y - exact, axis=1) / np.linalg.norm(exact, axis=1)
            assert err.max() < 1e-10
        assert vec_err(y[l], emu.Y) < 1e-10


@pytest.mark.parametrize("mode", ["mixed", "mixed_shifts"])
def test_mixed_precision_with_early_switch(sscg, prob, mode):
    """Switch to FP32 right away: reliable updates keep the seed residual honest, but the
    shifted solutions carry the FP32 rounding of the early, large updates (stated bound)."""
    case(f"{mode} precision switch_tol=1")
    U, A, V, z = prob
    prec = sscg.MIXED if mode == "mixed" else sscg.MIXED_SHIFTS
    y, r = solve(sscg, U, V, z, prec=prec, ru_interval=10, switch_tol=1.0)
    assert r.true_res.max() < 1e-4
    # the FP64 check after the solve names the inaccuracy: true residuals above
    # true_factor * tol (default 100 * 1e-12) give SSCG_EINACCURATE, not OK
    assert r.status == (sscg.OK if r.true_res.max() <= 100 * 1e-12 else sscg.EINACCURATE)
    for l in range(V.shape[0]):
        tr = solvers.true_residuals(lambda x: A @ x, V[l], z, y[l])
        assert np.abs(tr - r.true_res[l]).max() <= 1e-3 * tr.max()


def test_batch_equals_single(sscg):
    case("batched uneven problems")
    shapes = [((4, 4, 4, 4), 0.12, 16, 2), ((6, 4, 4, 4), 0.125, 12, 1), ((4, 4, 6, 6), 0.13, 8, 3)]
    ctxs, vs, zs, ys, singles = [], [], [], [], []
    for i, (dims, kappa, N, L) in enumerate(shapes):
        U = synth.gauge_field(dims, 0.5, 30 + i)
        Vh = synth.sources(int(np.prod(dims)), L, 40 + i).reshape(L, -1)
        z, _ = quad.line_nodes(N, 0.0, 0.2, 0.25)
        ys_single, r_single = solve(sscg, U, Vh, z, dims=dims, kappa=kappa)
        singles.append((ys_single, r_single))
        c = sscg.Context(dims, kappa)
        c.set_gauge(U)
        ctxs.append(c)
        vs.append(to_dev(Vh))
        zs.append(z)
        ys.append(to_dev(np.zeros((L, N, Vh.shape[1]))))
    res = sscg.batch_solve(ctxs, vs, zs, [0.0] * 3, ys)
    for (ys_single, r_single), y, r in zip(singles, ys, res):
        assert r.status == sscg.OK
        assert vec_err(to_host(y), ys_single) < 1e-11
        assert np.all(np.abs(r.iters - r_single.iters) <= 2)
        assert np.all(np.abs(r.conv_iter - r_single.conv_iter) <= 2)
        # FP64 rounding gap between the recursive and the true residual is about
        # eps * max_k ||r_k|| / ||v||; one of these sources passes a near-breakdown of
        # the indefinite seed where ||r_k|| peaks near 1e5 ||v|| (the oracle shows
        # 3e-11 on it), so the bar is 1e-10 rather than the tolerance itself
        assert r.true_res.max() < 1e-10


def test_zero_and_nan_sources_rejected(sscg, prob):
    case("zero / NaN source")
    U, A, V, z = prob
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    c.set_gauge(U)
    y = to_dev(np.zeros((1, len(z), CFG1.n)))
    for bad in (np.zeros((1, CFG1.n)), np.full((1, CFG1.n), np.nan)):
        with pytest.raises(sscg.SSCGError) as e:
            c.shifted_cg_solve(to_dev(bad.astype(complex)), z, 0.0, y)
        assert e.value.code == sscg.EINVAL


def test_empty_inputs_rejected(sscg, prob):
    """Empty inputs are argument errors at every entry point (no source, no shift, no
    moment), and an ss_eigs call that asks for no eigenpairs only counts them."""
    import torch
    case("empty inputs")
    U, A, V, z = prob
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    c.set_gauge(U)
    empty = torch.zeros(0, dtype=torch.complex128, device="cuda:0")
    for call in (lambda: c.apply_A(empty, empty),
                 lambda: c.shifted_cg_solve(empty, z, 0.0, empty),
                 lambda: c.shifted_cg_solve(to_dev(V[:1]), np.zeros(0, complex), 0.0, empty),
                 lambda: c.ss_moments(to_dev(np.zeros((1, len(z), CFG1.n))), len(z), np.zeros((0, len(z))),
                                      to_dev(np.zeros((1, CFG1.n))))):
        with pytest.raises(sscg.SSCGError) as e:
            call()
        assert e.value.code == sscg.EINVAL
    p = sscg.default_ss_params(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7)
    full = c.ss_eigs(p, to_dev(V[:2]), max_eigs=16)
    count = c.ss_eigs(p, to_dev(V[:2]), max_eigs=0)
    assert full.n_found > 0 and count.n_found == full.n_found
    c.close()


def test_no_gauge_is_a_state_error(sscg, prob):
    case("no gauge")
    U, A, V, z = prob
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    y = to_dev(np.zeros((1, len(z), CFG1.n)))
    with pytest.raises(sscg.SSCGError) as e:
        c.shifted_cg_solve(to_dev(V[:1]), z, 0.0, y)
    assert e.value.code == sscg.ESTATE


def test_maxiter_not_converged(sscg, prob):
    case("maxiter=1")
    U, A, V, z = prob
    y, r = solve(sscg, U, V[:1], z, maxiter=1)
    assert r.status == sscg.ENOTCONV
    assert np.all(r.conv_iter == -1) and r.iters[0] == 1


def test_breakdown_detected(sscg):
    case("breakdown B v = 0")
    dims, kappa = (4, 4, 4, 4), 0.125
    v = np.zeros((1, 256, 4, 3), dtype=complex)
    v[0, :, 0, 0] = 1.0
    y, r = solve(sscg, synth.unit_gauge(dims), v.reshape(1, -1), np.array([0.01j]), dims=dims, kappa=kappa)
    assert r.status == sscg.EBREAKDOWN
    assert r.iters[0] == 0


def test_shift_on_eigenvalue_only_that_shift_fails(sscg):
    case("shift on an eigenvalue")
    dims, kappa = (4, 4, 4, 4), 0.12
    v = synth.sources(256, 1, 7).reshape(1, -1)
    z = np.array([0.04 + 0j, 0.04 + 0.05j, -0.1 + 0.05j])
    y, r = solve(sscg, synth.unit_gauge(dims), v, z, dims=dims, kappa=kappa, maxiter=300)
    assert r.status == sscg.ENOTCONV
    assert r.conv_iter[0, 0] == -1 and r.conv_iter[0, 1] > 0 and r.conv_iter[0, 2] > 0
    assert r.true_res[0, 1] < 5e-12 and r.true_res[0, 2] < 5e-12


@pytest.mark.parametrize("mode", ["mixed", "mixed_shifts"])
def test_mixed_accuracy_check_status(sscg, prob, mode):
    """After a mixed-precision solve every shift's FP64 true residual is recomputed even
    when the caller does not ask for it: a bound below what the solve reached
    (true_factor 0.01, i.e. 1e-14) turns OK into SSCG_EINACCURATE, true_factor 0 only
    reports; the residuals it reports agree with the oracle's."""
    case(f"{mode} accuracy check status")
    U, A, V, z = prob
    prec = sscg.MIXED if mode == "mixed" else sscg.MIXED_SHIFTS
    y, r = solve(sscg, U, V, z, prec=prec, ru_interval=20, switch_tol=1e-6, true_factor=0.01)
    assert r.status == sscg.EINACCURATE
    for l in range(V.shape[0]):
        tr = solvers.true_residuals(lambda x: A @ x, V[l], z, y[l])
        assert np.abs(tr - r.true_res[l]).max() <= 1e-3 * tr.max()
    y2, r2 = solve(sscg, U, V, z, prec=prec, ru_interval=20, switch_tol=1e-6, true_factor=0.0)
    assert r2.status == sscg.OK
    assert vec_err(y2, y) < 1e-11   # separate contexts may tune other launch shapes


def test_ss_eigs_reports_mixed_true_residual(sscg, prob):
    """ss_eigs states the error of a mixed solve (largest FP64 true residual over all
    nodes and sources) and reports -1 for an FP64 solve, where it is not recomputed."""
    case("ss_eigs max_true_res")
    U, A, V, z = prob
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    c.set_gauge(U)
    vd = to_dev(V)
    out64 = c.ss_eigs(sscg.default_ss_params(gamma=0.0, rho=0.2, beta=0.25, N=16, M=8), vd, max_eigs=8)
    assert out64.info.max_true_res == -1.0
    p = sscg.default_ss_params(gamma=0.0, rho=0.2, beta=0.25, N=16, M=8,
                               solve=sscg.default_opts(prec=sscg.MIXED_SHIFTS, ru_interval=20))
    out = c.ss_eigs(p, vd, max_eigs=8)
    assert out.status == sscg.OK
    assert 0.0 < out.info.max_true_res < 1e-10


def test_seed_outside_the_spectrum(sscg, prob):
    """A seed shift outside the spectrum (sigma > 1 + 8 kappa >= ||A||) gives the same
    shifted iterates (they do not depend on the seed), so the same solutions and
    convergence iterations to within a few, with a seed residual that never grows
    and FP64 true residuals at least as close to the tolerance."""
    case("seed outside the spectrum")
    U, A, V, z = prob
    sigma = 1 + 8 * CFG1.kappa + 0.25
    y0, r0 = solve(sscg, U, V, z, sigma=0.0)
    y1, r1 = solve(sscg, U, V, z, sigma=sigma)
    assert r0.status == r1.status == sscg.OK
    # the centre seed's implicit residual lags by up to a few iterations after its
    # near-breakdowns; the definite seed never detects convergence later
    assert np.all(r1.conv_iter <= r0.conv_iter) and np.all(r0.conv_iter - r1.conv_iter <= 4)
    assert vec_err(y1, y0) < 1e-9
    assert r1.true_res.max() <= max(r0.true_res.max(), 2e-12)
    for l in range(V.shape[0]):
        assert solvers.true_residuals(lambda x: A @ x, V[l], z, y1[l]).max() < 5e-12
