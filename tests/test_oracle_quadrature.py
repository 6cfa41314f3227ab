"""Pins of the oracle's quadrature (Sec. 2.1 circle, Sec. 3 lines) and filter function eq. (3).

The line weights are checked against a 60-digit solve of the paper's own linear
system (not the closed form the oracle uses); the circle against the paper's
filter formula f_k(x) = x^k / (1 + x^N); the filter against its product form and
the identity f_k = x^k f_0 that makes the moment conditions the right ones.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as quad


def exact_weights(zeta):
    """Solve sum_j w_j zeta_j^(k-1) = delta_k0, k = 0..N-1, in 60-digit arithmetic."""
    mp.mp.dps = 60
    N = len(zeta)
    zs = [mp.mpc(complex(z).real, complex(z).imag) for z in zeta]
    Amat = mp.matrix(N, N)
    for k in range(N):
        for j in range(N):
            Amat[k, j] = zs[j] ** (k - 1)
    rhs = mp.matrix([1] + [0] * (N - 1))
    w = mp.lu_solve(Amat, rhs)
    return np.array([complex(w[j]) for j in range(N)])


@pytest.mark.parametrize("N,beta", [(4, 0.3), (8, 0.25), (16, 0.25), (32, 0.2), (64, 0.4)])
def test_line_weights_match_exact_solve(N, beta):
    z, zeta = quad.line_nodes(N, 0.0, 1.0, beta)
    w = quad.line_weights(zeta)
    we = exact_weights(zeta)
    assert np.abs(w - we).max() / np.abs(we).max() < 1e-13


@pytest.mark.parametrize("N", [8, 16, 32])
def test_circle_weights_satisfy_the_line_conditions(N):
    # the same moment conditions hold on the circle with w = zeta / N
    z, zeta = quad.circle_nodes(N, 0.3, 0.5)
    w = quad.circle_weights(zeta)
    for k in range(N):
        s = np.sum(w * zeta ** (k - 1))
        assert abs(s - (1.0 if k == 0 else 0.0)) < 1e-14
    assert np.allclose(quad.circle_weights(zeta), exact_weights(zeta), atol=1e-15)


def test_node_layout():
    N, gamma, rho, beta = 16, 0.1, 0.2, 0.25
    z, zeta = quad.line_nodes(N, gamma, rho, beta)
    assert np.allclose(zeta[0::2].imag, beta) and np.allclose(zeta[1::2].imag, -beta)
    assert np.allclose(zeta[1::2], zeta[0::2].conj())
    x = zeta[0::2].real
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.allclose(np.diff(x), 2.0 / (N // 2 - 1))
    assert np.allclose(z, gamma + rho * zeta)
    assert np.allclose(np.abs(z.imag), beta * rho)   # distance to the real axis is beta*rho


def product_filter(x, zeta):
    return np.prod(zeta[:, None] / (zeta[:, None] - np.asarray(x)[None, :]), axis=0)


@pytest.mark.parametrize("path", ["lines", "circle"])
def test_filter_product_form_and_power_shift(path):
    N = 32
    if path == "lines":
        _, zeta = quad.line_nodes(N, 0.0, 1.0, 0.3)
        w = quad.line_weights(zeta)
    else:
        _, zeta = quad.circle_nodes(N, 0.0, 1.0)
        w = quad.circle_weights(zeta)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1.6, 1.6, 40) + 1j * rng.uniform(-0.1, 0.1, 40)
    f0 = quad.filter_function(x, zeta, w, 0)
    assert np.abs(f0 - product_filter(x, zeta)).max() < 1e-11 * max(1.0, np.abs(f0).max())
    for k in (1, 5, N - 1):
        fk = quad.filter_function(x, zeta, w, k)
        assert np.abs(fk - x ** k * f0).max() < 1e-9 * max(1.0, np.abs(x ** k * f0).max())
    # beyond the conditions (k = N) a constant sum_j w_j zeta_j^(N-1) appears
    c = np.sum(w * zeta ** (N - 1))
    assert abs(c) > 1e-12
    fN = quad.filter_function(x, zeta, w, N)
    assert np.abs(fN - x ** N * f0 - c).max() < 1e-9 * max(1.0, np.abs(x ** N * f0).max())


@pytest.mark.parametrize("N", [16, 32])
def test_circle_filter_closed_form(N):
    # Sec. 2.1: on the unit circle f_k(x) = x^k / (1 + x^N)
    _, zeta = quad.circle_nodes(N, 0.0, 1.0)
    w = quad.circle_weights(zeta)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.5, 1.5, 30) + 1j * rng.uniform(-0.3, 0.3, 30)
    for k in (0, 3, N - 1):
        ref = x ** k / (1 + x ** N)
        assert np.abs(quad.filter_function(x, zeta, w, k) - ref).max() < 1e-11 * max(1, np.abs(ref).max())


@pytest.mark.parametrize("beta", [0.2, 0.6, 1.0, 1.4])
def test_line_filter_real_positive_and_normalised(beta):
    _, zeta = quad.line_nodes(32, 0.0, 1.0, beta)
    w = quad.line_weights(zeta)
    x = np.linspace(-3, 3, 61)
    f = product_filter(x, zeta)
    assert np.abs(f.imag).max() < 1e-15 * np.abs(f).max() + 1e-300
    assert np.all(f.real > 0)
    # f_0(0) = sum_j w_j / zeta_j = 1 (the k = 0 condition); rounding scales with sum |w_j / zeta_j|
    scale = np.sum(np.abs(w / zeta))
    assert abs(quad.filter_function(np.array([0.0]), zeta, w)[0] - 1) < 1e-14 * scale


def test_fig2_shapes():
    """Fig. 2: the circle filter has a plateau on [-1, 1]; the line filters have none
    and their fall-off from the centre is set by beta (slower for larger beta)."""
    _, zc = quad.circle_nodes(32, 0.0, 1.0)
    wc = quad.circle_weights(zc)
    xin = np.linspace(-0.7, 0.7, 15)
    assert np.abs(quad.filter_function(xin, zc, wc) - 1).max() < 1e-3
    assert abs(quad.filter_function(np.array([1.0]), zc, wc)[0] - 0.5) < 1e-12
    prev = None
    for beta in (0.2, 0.6, 1.0, 1.4):
        _, zl = quad.line_nodes(32, 0.0, 1.0, beta)
        f = product_filter(np.array([0.5, 1.0]), zl).real
        assert f[0] < 0.5            # no plateau
        if prev is not None:
            assert np.all(f > prev)  # broader for larger beta
        prev = f


def test_acceptance_interval():
    _, zeta = quad.line_nodes(32, 0.0, 1.0, 0.2)
    assert quad.acceptance_interval(zeta, 0.5, 0.1, 32) == pytest.approx((0.4, 0.6))
    lo, hi = quad.acceptance_interval(zeta, 0.0, 1.0, 16)
    assert (lo, hi) == pytest.approx((-7 / 15, 7 / 15))
    with pytest.raises(ValueError):
        quad.acceptance_interval(zeta, 0.0, 1.0, 6 + 1)


def test_adjacent_pairs_node_count_and_sharing():
    # Table 2: six pairs with N = 32, N' = 16 use 32 + 5 * 14 = 102 nodes (128 for four circles of 32)
    z_all, offsets, centres = quad.adjacent_pairs(32, 16, 6, 0.0, 0.02121, 0.2)
    assert z_all.size == 102 == 32 + 5 * (16 - 2)
    for p in range(6):
        zp = z_all[offsets[p]:offsets[p] + 32]
        z_ref, _ = quad.line_nodes(32, centres[p], 0.02121, 0.2)
        assert np.abs(zp - z_ref).max() < 1e-15
    # neighbouring acceptance rectangles share an edge and tile the whole range
    _, zeta = quad.line_nodes(32, 0.0, 1.0, 0.2)
    rects = [quad.acceptance_interval(zeta, c, 0.02121, 16) for c in centres]
    for (lo1, hi1), (lo2, hi2) in zip(rects, rects[1:]):
        assert hi1 == pytest.approx(lo2, abs=1e-15)
