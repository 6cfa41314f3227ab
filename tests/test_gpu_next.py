"""GPU parity of the extensions of the hot path named by the paper (Sec. 3-4).

* Adjacent line pairs sharing nodes (Sec. 3, end): one shifted CG over the
  N + (P-1)(N'-2) distinct nodes; per-pair extraction equals the oracle's and the
  dense spectrum (1e-10 relative, residual below 1e-8).
* The circle path C (Sec. 2.1, eq. 2): eigenvalues equal the oracle's and the dense
  spectrum; per-node convergence iterations grow as the node nears the real axis
  (the trend of Fig. 1).
* Rayleigh-Ritz versus Hankel (Sec. 2.1: RR is the more accurate of the two): on the
  same solves the RR residuals are below the Hankel ones and both certify their
  eigenvalues.
"""
import numpy as np
import pytest

import synth
from oracle import quadrature as quad
from oracle import solvers, ss, wilson
from tests.helpers import case, to_dev, to_host

pytestmark = pytest.mark.gpu
CFG1 = synth.CONFIGS["wilson4_fp64"]


@pytest.fixture(scope="module")
def f4(sscg):
    U = CFG1.gauge()
    A = wilson.hermitian_wilson(U, CFG1.dims, CFG1.kappa)
    lam = np.linalg.eigvalsh(A.toarray())
    c = sscg.Context(CFG1.dims, CFG1.kappa)
    c.set_gauge(U)
    return U, A, lam, c


def test_adjacent_pairs(sscg, f4):
    case("adjacent line pairs")
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 5).reshape(2, -1)
    N, Np, P, rho, beta, M, gamma = 16, 8, 3, 0.012, 0.25, 6, 0.225
    ref = ss.ss_eigs_adjacent(A, V, gamma, rho, beta, N, M, Np, P, rank_tol=1e-7)
    p = sscg.default_ss_params(gamma=gamma, rho=rho, beta=beta, N=N, M=M, Nprime=Np, npairs=P, rank_tol=1e-7)
    out = c.ss_eigs(p, to_dev(V), max_eigs=32)
    assert out.n_found == len(ref["lam"]) > 0
    assert np.all(np.abs(out.lam - ref["lam"]) <= 1e-10 * np.abs(ref["lam"]))
    lo = ref["centres"][0] - rho * (Np // 2 - 1) / (N // 2 - 1)
    hi = ref["centres"][-1] + rho * (Np // 2 - 1) / (N // 2 - 1)
    truth = lam[(lam >= lo) & (lam <= hi)]
    assert np.all(np.abs(out.lam - truth) <= 1e-10 * np.abs(truth))
    assert out.res.max() < 1e-8
    # one solve over the distinct nodes: 16 + 2 * 6 = 28 shifts
    nall = N + (P - 1) * (Np - 2)
    assert out.info.shift_updates <= 2 * nall * out.info.iters
    assert out.info.shift_updates > 2 * (nall - 1) * 10


def test_circle_path(sscg, f4):
    case("circle path")
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 6).reshape(2, -1)
    gamma, rho, N, M = 0.225, 0.03, 16, 8
    ref = ss.ss_eigs(A, V, gamma, rho, 0.25, N, M, path="circle", rank_tol=1e-7)
    p = sscg.default_ss_params(gamma=gamma, rho=rho, N=N, M=M, path=sscg.PATH_CIRCLE, rank_tol=1e-7)
    out = c.ss_eigs(p, to_dev(V), max_eigs=32)
    truth = lam[np.abs(lam - gamma) < rho]
    assert out.n_found == len(ref["lam"]) == len(truth)
    assert np.all(np.abs(out.lam - truth) <= 1e-10 * np.abs(truth))
    assert np.all(np.abs(out.lam - ref["lam"].real) <= 1e-10 * np.abs(truth))
    # the 1e-8 residual bar applies where the FP64 oracle itself meets it (with N = 16
    # and M = 8 the circle leaves some pairs just above it); elsewhere the GPU residual
    # must stay within twice the oracle's
    for r_gpu, r_ref in zip(out.res, ref["res"]):
        assert r_gpu <= max(1e-8, 2 * r_ref)


def test_circle_convergence_map(sscg, f4):
    """Fig. 1 trend: nodes closer to the real axis need more shifted-CG iterations."""
    case("circle convergence map")
    U, A, lam, c = f4
    z, zeta = quad.circle_nodes(32, 0.0, 0.2)
    v = CFG1.sources().reshape(1, -1)
    y = to_dev(np.zeros((1, 32, CFG1.n)))
    r = c.shifted_cg_solve(to_dev(v), z, 0.0, y)
    assert r.status == sscg.OK
    it = r.conv_iter[0]
    ref = solvers.shifted_cg(lambda x: A @ x, v[0], z, 0.0, 1e-12)
    assert np.all(np.abs(it - ref.conv_iter) <= 2)
    dist = np.abs(z.imag)
    order = np.argsort(dist)
    # the nodes nearest the axis take at least as many iterations as the farthest ones
    assert it[order[:4]].min() >= it[order[-4:]].max()
    # rank correlation between distance to the axis and iterations is negative
    rd = np.argsort(np.argsort(dist))
    ri = np.argsort(np.argsort(it))
    assert np.corrcoef(rd, ri)[0, 1] < -0.5


def test_rr_more_accurate_than_hankel(sscg, f4):
    case("RR vs Hankel")
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 7).reshape(2, -1)
    kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7)
    rr = c.ss_eigs(sscg.default_ss_params(method=sscg.RR, **kw), to_dev(V), max_eigs=16)
    hk = c.ss_eigs(sscg.default_ss_params(method=sscg.HANKEL, **kw), to_dev(V), max_eigs=16)
    assert rr.n_found == hk.n_found > 0
    assert np.median(rr.res) < np.median(hk.res)
    for out in (rr, hk):
        for l, r_ in zip(out.lam, out.res):
            assert np.abs(lam - l).min() <= r_ + 1e-13


@pytest.mark.parametrize("prec,P,pf,ub", [("fp64", 1, 0, 2), ("mixed_shifts", 1, 0, 2), ("fp64", 3, 0, 2),
                                         ("fp64", 1, 1, 1), ("fp64", 1, 1, 2), ("mixed_shifts", 1, 1, 2),
                                         ("fp64", 3, 1, 1), ("fp64", 1, 0, 4)])
def test_moments_in_loop(sscg, f4, monkeypatch, prec, P, pf, ub):
    """Moments summed inside the solve (no stored y_j) equal the stored-solution path
    and the oracle: same count, eigenvalues within 1e-10 relative, residuals below 1e-8
    (or twice the oracle's where N = 16, M = 8 leave the oracle itself above it). The
    update kernel runs with ub shifts per load group, with (pf = 1) or without the next
    group's loads issued ahead of the current group's stores."""
    case(f"in-loop moments {prec} P={P} pf={pf} ub={ub}")
    monkeypatch.setenv("SSCG_BLOCK", "0")  # the per-iteration form (pf and ub apply to it)
    monkeypatch.setenv("SSCG_MOMPF", str(pf))
    monkeypatch.setenv("SSCG_MOMUB", str(ub))
    _in_loop_vs_stored(sscg, f4, prec, P)


@pytest.mark.parametrize("prec,P,blk", [("fp64", 1, 4), ("fp64", 1, 8), ("fp64", 1, 16), ("fp64", 1, 32),
                                        ("mixed_shifts", 1, 8), ("mixed_shifts", 1, 32), ("fp64", 3, 8),
                                        ("mixed_shifts", 3, 16), ("fp64", 3, 24)])
def test_moments_in_loop_block(sscg, f4, monkeypatch, prec, P, blk):
    """Block form of the in-loop update (the recurrences of blk iterations composed
    into one linear map per shift and applied in one sweep over the directions, the
    seed residuals of the block kept in a ring): the same bar as the per-iteration
    form against the stored-solution path and the oracle."""
    case(f"in-loop moments block {blk} {prec} P={P}")
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    _in_loop_vs_stored(sscg, f4, prec, P)


@pytest.mark.parametrize("blk", [8, 16, 24, 32])
def test_moments_in_loop_block_cut_short(sscg, f4, monkeypatch, blk):
    """A solve stopped by the iteration limit (37, inside a block) in the block form:
    the sweep after the loop applies the partial block, so the moments, and the
    eigenvalues extracted from them, equal the per-iteration form's."""
    case(f"in-loop moments block {blk} cut short")
    U, A, lam, c = f4
    V = to_dev(synth.sources(CFG1.V, 2, 8).reshape(2, -1))
    # every Ritz value inside the rectangle is reported (no residual filter): the
    # truncated moments leave residuals far above any acceptance bar
    kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7, moments_in_loop=1, spur_tol=1e30)
    opts = sscg.default_opts(maxiter=37)
    keep = (sscg.EINVAL, sscg.ENOMEM, sscg.EDEVICE, sscg.ESTATE, sscg.EBREAKDOWN)
    monkeypatch.setenv("SSCG_BLOCK", "0")
    a = c.ss_eigs(sscg.default_ss_params(solve=opts, **kw), V, max_eigs=32, raise_on=keep)
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    b = c.ss_eigs(sscg.default_ss_params(solve=opts, **kw), V, max_eigs=32, raise_on=keep)
    assert a.info.solve_status == b.info.solve_status == sscg.ENOTCONV
    assert a.info.iters == b.info.iters == 37
    assert a.info.shift_updates == b.info.shift_updates
    assert a.info.rank == b.info.rank and a.n_found == b.n_found > 0
    assert np.all(np.abs(b.lam - a.lam) <= 1e-9 * np.abs(a.lam))
    assert np.all(np.abs(b.res - a.res) <= 1e-6 * a.res)


@pytest.mark.parametrize("blk", [8, 24])
def test_sweep_bytes_follow_the_shift_convergence(sscg, f4, monkeypatch, blk):
    """sscg_sweep_bytes (the benchmark's algorithmic bytes of the block sweep) equals the
    bytes the block form has to move, computed here from each shift's convergence
    iteration c_j, taken from a stored-solution solve of the same shifts: shift j is
    updated in iterations 0 .. c_j - 1 and freezes in the last. Per (source, block of
    iterations lo .. hi - 1): the moment kernel runs if a shift is updated in the block
    (c_j > lo) and reads those directions (v once in the first block), the blk residuals
    and the M moment sums and writes the sums; the direction kernel runs if a shift is
    still active at the block's end (c_j > hi), reads the same directions and the
    residuals and writes the active directions; 16 bytes per FP64 entry. The
    per-iteration form and stored solutions report 0."""
    import torch
    case(f"sweep bytes block {blk}")
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 8).reshape(2, -1)
    kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7)
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    out = c.ss_eigs(sscg.default_ss_params(moments_in_loop=1, **kw), to_dev(V), max_eigs=32)
    got = c.sweep_bytes()
    z, _, _ = sscg.quad_lines(kw["N"], kw["gamma"], kw["rho"], kw["beta"])
    y = torch.zeros((V.shape[0], kw["N"], V.shape[1]), dtype=torch.complex128, device="cuda:0")
    r = c.shifted_cg_solve(to_dev(V), z, kw["gamma"], y, sscg.default_ss_params().solve)
    assert r.status == sscg.OK and int(r.conv_iter.sum()) == out.info.shift_updates
    n, B, M, d = V.shape[1], blk, kw["M"], 16
    want = 0
    for l in range(V.shape[0]):
        cj = r.conv_iter[l].astype(np.int64)
        for b in range(-(-int(r.iters[l]) // B)):
            lo, hi = b * B, (b + 1) * B
            n_any, n_st = int((cj > lo).sum()), int((cj > hi).sum())
            rd = 1 if b == 0 else n_any
            if n_any:
                want += (16 * B + 32 * M + d * rd) * n
            if n_st:
                want += (16 * B + d * rd + d * n_st) * n
    assert got == want
    monkeypatch.setenv("SSCG_BLOCK", "0")
    c.ss_eigs(sscg.default_ss_params(moments_in_loop=1, **kw), to_dev(V), max_eigs=32)
    assert c.sweep_bytes() == 0


def _in_loop_vs_stored(sscg, f4, prec, P):
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 8).reshape(2, -1)
    pr = {"fp64": sscg.FP64, "mixed_shifts": sscg.MIXED_SHIFTS}[prec]
    opts = sscg.default_opts(prec=pr, switch_tol=1e-6, ru_interval=20)
    if P == 1:
        kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7)
        ref = ss.ss_eigs(A, V, kw["gamma"], kw["rho"], kw["beta"], kw["N"], kw["M"], rank_tol=1e-7)
    else:
        kw = dict(gamma=0.225, rho=0.012, beta=0.25, N=16, M=6, Nprime=8, npairs=3, rank_tol=1e-7)
        ref = ss.ss_eigs_adjacent(A, V, 0.225, 0.012, 0.25, 16, 6, 8, 3, rank_tol=1e-7)
    stored = c.ss_eigs(sscg.default_ss_params(solve=opts, **kw), to_dev(V), max_eigs=32)
    fused = c.ss_eigs(sscg.default_ss_params(solve=opts, moments_in_loop=1, **kw), to_dev(V), max_eigs=32)
    assert fused.n_found == stored.n_found == len(ref["lam"]) > 0
    assert np.all(np.abs(fused.lam - stored.lam) <= 1e-11 * np.abs(stored.lam))
    assert np.all(np.abs(fused.lam - np.real(ref["lam"])) <= 1e-10 * np.abs(fused.lam))
    # residual bar as for the circle: 1e-8 where the FP64 oracle meets it, else twice its own
    assert np.all(fused.res <= np.maximum(1e-8, 2 * ref["res"]))
    assert fused.info.iters == stored.info.iters
    assert fused.info.shift_updates == stored.info.shift_updates
    # eigenvectors agree up to phase
    Xf, Xs = to_host(fused.X), to_host(stored.X)
    for k in range(fused.n_found):
        ov = abs(np.vdot(Xf[k].ravel(), Xs[k].ravel()))
        assert ov > 1 - 1e-9


@pytest.mark.parametrize("prec,blk", [("fp64", 0), ("mixed_shifts", 0), ("fp64", 8), ("mixed_shifts", 4)])
def test_moments_in_loop_ragged_chunks(sscg, monkeypatch, prec, blk):
    """In-loop moments on a lattice whose vector length n = 12 V = 1620 is not a
    multiple of 64: the shift directions are stored in 64-entry chunks with a padded
    last chunk. Eigenpairs equal the stored-solution path and the dense spectrum
    (per-iteration form, blk = 0, and block form)."""
    case(f"in-loop moments ragged chunks {prec} block {blk}")
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    dims, kappa = (3, 3, 3, 5), 0.12
    U = synth.gauge_field(dims, 0.3, 11)
    A = wilson.hermitian_wilson(U, dims, kappa)
    lam = np.linalg.eigvalsh(A.toarray())
    V = synth.sources(int(np.prod(dims)), 2, 12).reshape(2, -1)
    # a window around the smallest positive eigenvalue holding a few eigenvalues
    pos = np.sort(lam[lam > 0])
    gamma, rho = float(0.5 * (pos[0] + pos[3])), float(0.5 * (pos[3] - pos[0]) + 0.25 * (pos[4] - pos[3]))
    inside = lam[(lam > gamma - rho) & (lam < gamma + rho)]
    c = sscg.Context(dims, kappa)
    c.set_gauge(U)
    pr = {"fp64": sscg.FP64, "mixed_shifts": sscg.MIXED_SHIFTS}[prec]
    opts = sscg.default_opts(prec=pr, switch_tol=1e-6, ru_interval=20)
    kw = dict(gamma=gamma, rho=rho, beta=0.25, N=16, M=8, rank_tol=1e-7)
    stored = c.ss_eigs(sscg.default_ss_params(solve=opts, **kw), to_dev(V), max_eigs=16)
    fused = c.ss_eigs(sscg.default_ss_params(solve=opts, moments_in_loop=1, **kw), to_dev(V), max_eigs=16)
    c.close()
    assert fused.n_found == stored.n_found == len(inside) > 0
    assert np.all(np.abs(fused.lam - stored.lam) <= 1e-11 * np.abs(stored.lam))
    assert np.all(np.abs(np.sort(fused.lam) - np.sort(inside)) <= 1e-10 * np.abs(np.sort(inside)))
    assert np.all(fused.res < 1e-8)


def test_moments_in_loop_rejects(sscg, f4):
    case("in-loop moments argument errors")
    U, A, lam, c = f4
    V = to_dev(synth.sources(CFG1.V, 2, 8).reshape(2, -1))
    base = dict(gamma=0.225, rho=0.03, N=16, M=8, moments_in_loop=1)
    for kw in (dict(method=sscg.HANKEL, N=48, M=20), dict(M=33), dict(M=12, npairs=3, Nprime=8),
               dict(solve=sscg.default_opts(prec=sscg.MIXED))):
        with pytest.raises(sscg.SSCGError) as e:
            c.ss_eigs(sscg.default_ss_params(**{**base, **kw}), V, max_eigs=8)
        assert e.value.code == sscg.EINVAL


@pytest.mark.parametrize("in_loop,blk", [(0, 0), (1, 0), (1, 8)])
def test_weighted_tolerance(sscg, f4, monkeypatch, in_loop, blk):
    """Moment-weighted stopping on the GPU equals the oracle's: the same shift-update
    count (each node's convergence iteration within 2), eigenvalues within 1e-10
    (stored solutions, in-loop moments, and their block form, where the shifts freeze
    at different iterations inside a block)."""
    case(f"weighted tolerance in_loop={in_loop} block {blk}")
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 9).reshape(2, -1)
    kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7)
    ref = ss.ss_eigs(A, V, kw["gamma"], kw["rho"], kw["beta"], kw["N"], kw["M"], rank_tol=1e-7,
                     weighted_tol=True)
    out = c.ss_eigs(sscg.default_ss_params(weighted_tol=1, moments_in_loop=in_loop, **kw), to_dev(V),
                    max_eigs=32)
    su_ref = sum(int(np.where(r.conv_iter >= 0, r.conv_iter, r.iters).sum()) for r in ref["runs"])
    assert abs(out.info.shift_updates - su_ref) <= 2 * kw["N"] * 2
    plain = c.ss_eigs(sscg.default_ss_params(**kw), to_dev(V), max_eigs=32)
    assert out.info.shift_updates < plain.info.shift_updates
    assert out.n_found == len(ref["lam"]) > 0
    assert np.all(np.abs(out.lam - np.real(ref["lam"])) <= 1e-10 * np.abs(out.lam))
    assert np.all(out.res <= np.maximum(1e-8, 2 * ref["res"]))


@pytest.mark.parametrize("blk", [0, 16])
def test_hankel_with_moments_in_loop(sscg, f4, monkeypatch, blk):
    """Hankel extraction from 2M moments summed inside the solve (block moments
    V^H s_k formed from them) equals the stored-solution Hankel and the oracle's
    (per-iteration form, blk = 0, and block form)."""
    case(f"Hankel with in-loop moments block {blk}")
    monkeypatch.setenv("SSCG_BLOCK", str(blk))
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 7).reshape(2, -1)
    kw = dict(gamma=0.225, rho=0.03, beta=0.25, N=16, M=8, rank_tol=1e-7, method=sscg.HANKEL)
    ref = ss.ss_eigs(A, V, 0.225, 0.03, 0.25, 16, 8, method="hankel", rank_tol=1e-7)
    stored = c.ss_eigs(sscg.default_ss_params(**kw), to_dev(V), max_eigs=16)
    fused = c.ss_eigs(sscg.default_ss_params(moments_in_loop=1, **kw), to_dev(V), max_eigs=16)
    assert fused.n_found == stored.n_found == len(ref["lam"]) > 0
    assert np.all(np.abs(fused.lam - stored.lam) <= 1e-10 * np.abs(stored.lam))
    assert np.all(np.abs(fused.lam - np.real(ref["lam"])) <= 1e-10 * np.abs(fused.lam))
    assert np.all(fused.res <= np.maximum(1e-8, 2 * ref["res"]))


def test_smaller_beta_costs_more_matvecs(sscg, f4):
    """Sec. 3 trend: lines closer to the real axis (smaller beta) need more seed
    iterations (matrix-vector products): on the GPU and in the oracle the seed
    iterations fall strictly as beta grows, and agree within 10 % (the last shifts to
    converge sit on slowly falling residual curves, where rounding moves the crossing
    of the tolerance by tens of iterations). (The paper's companion trend, higher
    accuracy at smaller beta, is not monotone on this synthetic field with N = 16,
    M = 8, and is not asserted.)"""
    case("beta trend of the seed iterations")
    U, A, lam, c = f4
    V = synth.sources(CFG1.V, 2, 5).reshape(2, -1)
    its, refs = [], []
    for beta in (0.1, 0.25, 0.5, 1.0):
        ref = ss.ss_eigs(A, V, 0.225, 0.03, beta, 16, 8, rank_tol=1e-7)
        out = c.ss_eigs(sscg.default_ss_params(gamma=0.225, rho=0.03, beta=beta, N=16, M=8, rank_tol=1e-7),
                        to_dev(V), max_eigs=16)
        ref_it = sum(r.iters for r in ref["runs"])
        assert abs(out.info.seed_iters - ref_it) <= 0.1 * ref_it
        assert out.n_found == len(ref["lam"])
        its.append(out.info.seed_iters)
        refs.append(ref_it)
    for seq in (its, refs):
        assert all(a > b for a, b in zip(seq, seq[1:]))
