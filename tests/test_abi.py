"""The C-ABI library loads, exports every function include/sscg.h declares, and its
host-only entry points (quadrature, small Hermitian eigensolver, argument checks)
agree with the oracle. No device is needed."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

from oracle import quadrature as quad

HEADER = Path(__file__).resolve().parent.parent / "include" / "sscg.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sscg_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sscg_set_gauge", "sscg_apply_A", "sscg_shifted_cg_solve", "sscg_ss_moments",
                     "sscg_ss_eigs"):
        assert required in names


def test_library_exports_every_declared_symbol(sscg):
    lib = sscg.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sscg.EXPORTS)


def test_exports_are_c_linkage(sscg):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", str(sscg.LIB_PATH)], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sscg_\w+)", out))
    assert set(declared_functions()) <= exported


@pytest.mark.parametrize("N,gamma,rho,beta", [(16, 0.0, 0.2, 0.25), (32, 0.1, 0.05, 0.4), (64, 0.0, 0.05, 0.4)])
def test_quad_lines_matches_oracle(sscg, N, gamma, rho, beta):
    z, ze, w = sscg.quad_lines(N, gamma, rho, beta)
    z2, ze2 = quad.line_nodes(N, gamma, rho, beta)
    w2 = quad.line_weights(ze2)
    assert np.abs(z - z2).max() < 1e-15
    assert np.abs(w - w2).max() / np.abs(w2).max() < 1e-13


def test_quad_circle_matches_oracle(sscg):
    z, ze, w = sscg.quad_circle(32, 0.1, 0.3)
    z2, ze2 = quad.circle_nodes(32, 0.1, 0.3)
    assert np.abs(z - z2).max() < 1e-15
    assert np.abs(w - quad.circle_weights(ze2)).max() < 1e-16


def test_quad_rejects_bad_arguments(sscg):
    with pytest.raises(sscg.SSCGError):
        sscg.quad_lines(7, 0.0, 0.1, 0.2)
    with pytest.raises(sscg.SSCGError):
        sscg.quad_lines(16, 0.0, -0.1, 0.2)


@pytest.mark.parametrize("n", [1, 2, 7, 40, 130])
def test_herm_eig(sscg, n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = B + B.conj().T
    ev, V = sscg.herm_eig(A)
    assert np.abs(ev - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1, np.abs(ev).max())
    assert np.abs(A @ V - V * ev).max() < 1e-11 * max(1, np.abs(ev).max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("scale", [1e-100, 1e100])
def test_herm_eig_scaled(sscg, scale):
    rng = np.random.default_rng(5)
    B = rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24))
    A = (B + B.conj().T) * scale
    ev, V = sscg.herm_eig(A)
    ref = np.linalg.eigvalsh(A)
    assert np.abs(ev - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(V.conj().T @ V - np.eye(24)).max() < 1e-12


def test_herm_eig_degenerate(sscg):
    A = np.diag([1.0, 1.0, 2.0, 2.0, 2.0]).astype(complex)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((5, 5)) + 0j)
    ev, V = sscg.herm_eig(Q @ A @ Q.conj().T)
    assert np.allclose(ev, [1, 1, 2, 2, 2], atol=1e-14)


def test_create_without_device_fails_cleanly(sscg):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(sscg.SSCGError) as e:
        sscg.Context((4, 4, 4, 4), 0.12)
    assert e.value.code in (sscg.EDEVICE, sscg.EINVAL)


def test_create_rejects_bad_lattice(sscg):
    with pytest.raises(sscg.SSCGError) as e:
        sscg.Context((4, 0, 4, 4), 0.12)
    assert e.value.code == sscg.EINVAL
    with pytest.raises(sscg.SSCGError) as e:
        sscg.Context((4, 4, 4, 4), 0.12, r=0.5)
    assert e.value.code == sscg.EINVAL


def test_struct_layouts_match_header(sscg, tmp_path):
    """The ctypes mirrors of the option, parameter and info structs have the size and
    field offsets the C header gives them (compiled with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"sscg_solve_opts": sscg.SolveOpts, "sscg_ss_params": sscg.SSParams, "sscg_ss_info": sscg.SSInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("n", [1, 2, 256])
def test_herm_eig_sizes(sscg, n):
    """Smallest sizes and the largest projected matrix the extraction forms (M L <= 256),
    with a graded spectrum spanning ten orders of magnitude."""
    rng = np.random.default_rng(100 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.sort(np.geomspace(1e-10, 1.0, n) * np.where(np.arange(n) % 2, -1.0, 1.0))
    A = (Q * lam) @ Q.conj().T
    ev, V = sscg.herm_eig(A)
    assert np.abs(ev - lam).max() < 1e-13
    assert np.abs(A @ V - V * ev).max() < 1e-13
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12


def test_herm_eig_already_split(sscg):
    """A tridiagonal input whose off-diagonal entries are below the deflation threshold
    in some places (the iteration splits it into independent blocks)."""
    n = 40
    d = np.linspace(-1.0, 1.0, n)
    e = np.full(n - 1, 0.3)
    e[::7] = 1e-18
    A = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ev, V = sscg.herm_eig(A.astype(complex))
    assert np.abs(ev - np.linalg.eigvalsh(A)).max() < 1e-14
    assert np.abs(A @ V - V * ev).max() < 1e-14
