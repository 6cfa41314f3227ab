"""Pins of the oracle's Wilson matrix A = gamma5 (I - kappa D) (Sec. 4) and of the SU(3) inputs.

Each check compares the explicit sparse assembly with something computed another
way: the Clifford algebra, the Hermiticity that gamma5-hermiticity implies, the
plane-wave spectrum of the free field, the gauge covariance of the hopping term,
and norm bounds. Mutations planted in the oracle at the end show that a wrong
sign, a missing adjoint or a wrong basis fails at least one pin.
"""
import numpy as np
import pytest

import synth
from oracle import wilson


def test_clifford_algebra_and_gamma5():
    g = wilson.gamma_matrices()
    for a in range(5):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(5):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * np.eye(4) * (a == b))
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))


def test_su3_links():
    U = synth.gauge_field((4, 4, 4, 4), 0.7, 3)
    UU = np.einsum("mvji,mvjk->mvik", U.conj(), U)
    assert np.abs(UU - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    G = synth.gell_mann()
    assert np.allclose(np.einsum("aij,bji->ab", G, G), 2 * np.eye(8))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 3), (3, 4, 5, 2)])
def test_structure_and_hermiticity(dims):
    U = synth.gauge_field(dims, 0.5, 1)
    A = wilson.hermitian_wilson(U, dims, 0.13)
    n = 12 * int(np.prod(dims))
    assert A.shape == (n, n)
    if min(dims) >= 3:
        # 1 diagonal + 8 hops x 2 spin entries x 3 colours per row (with an extent
        # of 2 the forward and backward neighbours coincide and entries merge)
        assert np.all(np.diff(A.indptr) == 49)
    assert abs(A - A.getH()).max() == 0.0


def test_paper_dimensions():
    # Sec. 4: 12^3 x 24 lattice gives a 497,664-dimensional matrix
    assert 12 * 12 ** 3 * 24 == 497664


def test_free_field_spectrum_4444():
    dims, kappa = (4, 4, 4, 4), 0.12
    A = wilson.hermitian_wilson(synth.unit_gauge(dims), dims, kappa)
    ev = np.linalg.eigvalsh(A.toarray())
    ff = wilson.free_field_spectrum(dims, kappa)
    assert np.abs(ev - ff).max() < 1e-13
    inside = ev[np.abs(ev) <= 0.2]
    assert len(inside) == 12 and np.allclose(np.sort(inside), [-0.04] * 6 + [0.04] * 6, atol=1e-13)
    # next momentum p = (pi/2, 0, 0, 0): m = 1 - 2 kappa (0 + 3) = 0.28, |s| = 2 kappa
    assert np.sort(np.abs(ev))[12] == pytest.approx(np.hypot(0.28, 0.24), abs=1e-13)


def test_free_field_spectrum_asymmetric():
    dims, kappa = (2, 3, 4, 5), 0.09
    A = wilson.hermitian_wilson(synth.unit_gauge(dims), dims, kappa)
    ev = np.linalg.eigvalsh(A.toarray())
    assert np.abs(ev - wilson.free_field_spectrum(dims, kappa)).max() < 1e-13


def gauge_transform(U, Om, dims):
    out = np.empty_like(U)
    for mu in range(4):
        fwd = wilson.neighbour(dims, mu, +1)
        out[mu] = Om @ U[mu] @ Om[fwd].conj().transpose(0, 2, 1)
    return out


def test_gauge_covariance():
    dims, kappa = (4, 4, 2, 4), 0.11
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 0.6, 2)
    Om = synth.random_gauge_transform(V, 9)
    A = wilson.hermitian_wilson(U, dims, kappa).toarray()
    A2 = wilson.hermitian_wilson(gauge_transform(U, Om, dims), dims, kappa).toarray()
    # block-diagonal Omega acting on colour: (I4 (x) Omega(x)) per site
    Ob = np.zeros((12 * V, 12 * V), dtype=complex)
    for s in range(V):
        Ob[12 * s:12 * s + 12, 12 * s:12 * s + 12] = np.kron(np.eye(4), Om[s])
    assert np.abs(A2 - Ob @ A @ Ob.conj().T).max() < 1e-13


def test_norm_bounds():
    dims, kappa = (3, 3, 3, 4), 0.11
    A = wilson.hermitian_wilson(synth.gauge_field(dims, 0.9, 4), dims, kappa)
    ev = np.linalg.eigvalsh(A.toarray())
    assert np.abs(ev).max() <= 1 + 8 * kappa
    assert np.abs(ev).min() >= 1 - 8 * kappa


# ---- planted mistakes -------------------------------------------------------

def pins_pass(monkeypatch_build):
    # every extent >= 3, so forward and backward neighbours differ in each direction
    dims, kappa = (3, 3, 3, 4), 0.12
    A = monkeypatch_build(synth.gauge_field(dims, 0.4, 0), dims, kappa)
    herm = abs(A - A.getH()).max() < 1e-14
    A1 = monkeypatch_build(synth.unit_gauge(dims), dims, kappa)
    ev = np.linalg.eigvalsh(A1.toarray())
    ff = ev.shape == wilson.free_field_spectrum(dims, kappa).shape and \
        np.abs(ev - wilson.free_field_spectrum(dims, kappa)).max() < 1e-12
    return herm and ff


def test_pins_pass_on_the_oracle():
    assert pins_pass(wilson.hermitian_wilson)


def test_planted_wrong_gamma5(monkeypatch):
    orig = wilson.gamma_matrices

    def bad():
        g = orig()
        g[4] = np.diag([1, -1, 1, -1]).astype(complex)
        return g
    monkeypatch.setattr(wilson, "gamma_matrices", bad)
    assert not pins_pass(wilson.hermitian_wilson)


def test_planted_missing_adjoint(monkeypatch):
    monkeypatch.setattr(wilson, "adjoint", lambda M: M)
    assert not pins_pass(wilson.hermitian_wilson)


def test_planted_transposed_link(monkeypatch):
    monkeypatch.setattr(wilson, "adjoint", lambda M: M.swapaxes(-1, -2))
    assert not pins_pass(wilson.hermitian_wilson)


def test_planted_wrong_neighbour(monkeypatch):
    orig = wilson.neighbour
    monkeypatch.setattr(wilson, "neighbour", lambda dims, mu, step: orig(dims, mu, abs(step)))
    assert not pins_pass(wilson.hermitian_wilson)


def test_global_gamma_sign_is_a_basis_change(monkeypatch):
    orig = wilson.gamma_matrices

    def bad():
        g = orig()
        g[:4] = -g[:4]   # (r + gamma) forward and (r - gamma) backward
        g[4] = orig()[4]
        return g
    monkeypatch.setattr(wilson, "gamma_matrices", bad)
    # Flipping all four gamma_mu keeps gamma5 and is a change of basis: these
    # pins cannot see it, so the hop-direction convention (1 - gamma_mu forward)
    # is fixed by the element-by-element GPU parity tests instead.
    assert pins_pass(wilson.hermitian_wilson)


def test_apply_rows_matches_explicit_matrix():
    dims, kappa = (4, 3, 5, 4), 0.13
    U = synth.gauge_field(dims, 0.6, 5)
    A = wilson.hermitian_wilson(U, dims, kappa)
    x = synth.sources(int(np.prod(dims)), 1, 2).reshape(-1)
    sites = [0, 7, 59, 239, 120]
    got = wilson.apply_rows(U, dims, kappa, x, sites)
    full = (A @ x).reshape(-1, 12)
    assert np.abs(got - full[sites]).max() < 1e-14
