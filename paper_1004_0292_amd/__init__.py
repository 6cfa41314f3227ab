"""Python binding of libsscg (the C-ABI in include/sscg.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch tensors
(device memory) and numpy arrays (host memory) into the pointers and sizes the
C functions take, and turns status codes into exceptions. There is no fallback:
if libsscg.so is missing or fails to load, importing the binding's functions
raises.

Names follow the C entry points: set_gauge, apply_A, shifted_cg_solve,
ss_moments, ss_eigs, quad_lines, quad_circle, batch_solve.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("SSCG_LIB", _PKG / "libsscg.so"))

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, ESTATE, EINACCURATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED, MIXED_SHIFTS = 0, 1, 2
PATH_LINES, PATH_CIRCLE = 0, 1
RR, HANKEL = 0, 1
_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOTCONV: "ENOTCONV",
           EBREAKDOWN: "EBREAKDOWN", ESTATE: "ESTATE", EINACCURATE: "EINACCURATE"}


class SSCGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("prec", C.c_int32),
                ("ru_interval", C.c_int32), ("poll_every", C.c_int32), ("switch_tol", C.c_double),
                ("use_graph", C.c_int32), ("pad", C.c_int32), ("true_factor", C.c_double)]


class SSParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("rho", C.c_double), ("beta", C.c_double),
                ("N", C.c_int32), ("M", C.c_int32), ("Nprime", C.c_int32), ("path", C.c_int32),
                ("method", C.c_int32), ("rank_tol", C.c_double), ("spur_tol", C.c_double),
                ("solve", SolveOpts), ("npairs", C.c_int32), ("moments_in_loop", C.c_int32),
                ("weighted_tol", C.c_int32), ("seed_mode", C.c_int32)]


class SSInfo(C.Structure):
    _fields_ = [("rank", C.c_int32), ("n_candidates", C.c_int32), ("iters", C.c_int32),
                ("solve_status", C.c_int32), ("t_solve", C.c_double), ("t_moments", C.c_double),
                ("t_extract", C.c_double), ("shift_updates", C.c_int64), ("matvecs", C.c_int64),
                ("shift_updates_fp32", C.c_int64), ("seed_iters", C.c_int64), ("seed_iters_fp32", C.c_int64),
                ("switch_iter", C.c_int32), ("pad", C.c_int32), ("max_true_res", C.c_double),
                ("extract_bytes", C.c_int64)]


EXPORTS = ["sscg_create", "sscg_destroy", "sscg_last_error", "sscg_global_error", "sscg_set_gauge",
           "sscg_apply_A", "sscg_apply_A_noalloc", "sscg_default_opts", "sscg_shifted_cg_solve", "sscg_ss_moments",
           "sscg_default_ss_params", "sscg_ss_eigs", "sscg_quad_lines", "sscg_quad_circle",
           "sscg_batch_solve", "sscg_herm_eig", "sscg_set_profiling", "sscg_stage_times",
           "sscg_stage_launches", "sscg_sweep_bytes"]

_lib = None


def lib() -> C.CDLL:
    """Load libsscg.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1004_0292_amd.build`")
    L = C.CDLL(str(LIB_PATH))
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    pd, pi = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    L.sscg_create.argtypes = [C.POINTER(vp), pi, dbl, dbl, i32, vp]
    L.sscg_destroy.argtypes = [vp]
    L.sscg_destroy.restype = None
    L.sscg_last_error.argtypes = [vp]
    L.sscg_last_error.restype = C.c_char_p
    L.sscg_global_error.argtypes = []
    L.sscg_global_error.restype = C.c_char_p
    L.sscg_set_gauge.argtypes = [vp, pd, i32]
    L.sscg_apply_A.argtypes = [vp, vp, vp, i32, i32]
    L.sscg_apply_A_noalloc.argtypes = [vp, vp, vp, i32, i32]
    L.sscg_default_opts.argtypes = [C.POINTER(SolveOpts)]
    L.sscg_default_opts.restype = None
    L.sscg_shifted_cg_solve.argtypes = [vp, vp, i32, pd, i32, dbl, C.POINTER(SolveOpts), vp, pi, pd, pi]
    L.sscg_ss_moments.argtypes = [vp, vp, i32, i32, pd, i32, vp]
    L.sscg_default_ss_params.argtypes = [C.POINTER(SSParams)]
    L.sscg_default_ss_params.restype = None
    L.sscg_ss_eigs.argtypes = [vp, C.POINTER(SSParams), vp, i32, i32, pd, vp, pd, pi, C.POINTER(SSInfo)]
    L.sscg_quad_lines.argtypes = [i32, dbl, dbl, dbl, pd, pd, pd]
    L.sscg_quad_circle.argtypes = [i32, dbl, dbl, pd, pd, pd]
    L.sscg_batch_solve.argtypes = [C.POINTER(vp), i32, C.POINTER(vp), pi, C.POINTER(pd), pi, pd,
                                   C.POINTER(SolveOpts), C.POINTER(vp), C.POINTER(pi), C.POINTER(pd),
                                   C.POINTER(pi)]
    L.sscg_herm_eig.argtypes = [i32, pd, pd, pd]
    L.sscg_set_profiling.argtypes = [vp, i32]
    L.sscg_stage_times.argtypes = [vp, pd, C.POINTER(C.c_int64)]
    L.sscg_stage_launches.argtypes = [vp, C.POINTER(C.c_int64)]
    L.sscg_sweep_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
    _lib = L
    return L


def _pd(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _cplx_host(a) -> np.ndarray:
    """complex128 host array as a contiguous float64 view (interleaved re, im)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a.view(np.float64)


def _check_dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous complex128 CUDA/HIP tensor")
    return C.c_void_p(t.data_ptr())


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().sscg_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_ss_params(**kw) -> SSParams:
    p = SSParams()
    lib().sscg_default_ss_params(C.byref(p))
    solve = kw.pop("solve", None)
    for k, v in kw.items():
        setattr(p, k, v)
    if solve is not None:
        p.solve = solve
    return p


def quad_lines(N, gamma, rho, beta):
    """Nodes z, normalised nodes zeta and weights w on the lines L+- (complex128 [N] each)."""
    z, ze, w = (np.zeros(2 * N) for _ in range(3))
    rc = lib().sscg_quad_lines(N, gamma, rho, beta, _pd(z), _pd(ze), _pd(w))
    if rc != OK:
        raise SSCGError(rc, lib().sscg_global_error().decode())
    return z.view(np.complex128), ze.view(np.complex128), w.view(np.complex128)


def quad_circle(N, gamma, rho):
    z, ze, w = (np.zeros(2 * N) for _ in range(3))
    rc = lib().sscg_quad_circle(N, gamma, rho, _pd(z), _pd(ze), _pd(w))
    if rc != OK:
        raise SSCGError(rc, lib().sscg_global_error().decode())
    return z.view(np.complex128), ze.view(np.complex128), w.view(np.complex128)


def herm_eig(A: np.ndarray):
    """Eigen-decomposition of a small Hermitian matrix by the library's host routine."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    a = _cplx_host(np.asfortranarray(A).ravel(order="F"))
    ev = np.zeros(n)
    V = np.zeros(2 * n * n)
    rc = lib().sscg_herm_eig(n, _pd(a), _pd(ev), _pd(V))
    if rc != OK:
        raise SSCGError(rc, lib().sscg_global_error().decode())
    return ev, V.view(np.complex128).reshape(n, n, order="F")


@dataclass
class SolveResult:
    status: int
    conv_iter: np.ndarray   # [nsrc][nshift]
    true_res: np.ndarray    # [nsrc][nshift]
    iters: np.ndarray       # [nsrc]


@dataclass
class EigResult:
    status: int
    lam: np.ndarray
    res: np.ndarray
    n_found: int
    X: object               # torch tensor [k][V][4][3] or None
    info: SSInfo


class Context:
    """One lattice on one device (sscg_create / sscg_destroy)."""

    def __init__(self, dims, kappa, r=1.0, device=0, stream=None):
        L = lib()
        self._h = C.c_void_p()
        d = np.asarray(dims, dtype=np.int32)
        s = C.c_void_p(stream) if stream is not None else None
        rc = L.sscg_create(C.byref(self._h), _pi(d), float(kappa), float(r), int(device), s)
        if rc != OK:
            raise SSCGError(rc, L.sscg_global_error().decode())
        self.dims = tuple(int(x) for x in dims)
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V
        self.kappa = kappa
        self.device = device

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sscg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, rc):
        raise SSCGError(rc, lib().sscg_last_error(self._h).decode())

    def set_gauge(self, U: np.ndarray, link_reals: int = 18):
        U = np.asarray(U, dtype=np.complex128)
        if U.shape != (4, self.V, 3, 3):
            raise ValueError(f"gauge must have shape (4, {self.V}, 3, 3)")
        u = _cplx_host(U)
        rc = lib().sscg_set_gauge(self._h, _pd(u), int(link_reals))
        if rc != OK:
            self._raise(rc)

    def apply_A(self, x, y, prec=FP64):
        nsrc = x.numel() // self.n
        if x.numel() != nsrc * self.n or y.numel() != x.numel():
            raise ValueError("x and y must hold nsrc * 12V entries")
        rc = lib().sscg_apply_A(self._h, _check_dev(x, "x"), _check_dev(y, "y"), nsrc, prec)
        if rc != OK:
            self._raise(rc)

    def apply_A_noalloc(self, x, y, prec=FP64):
        """y = A x with no device allocation (the library's static staging array)."""
        nsrc = x.numel() // self.n
        if x.numel() != nsrc * self.n or y.numel() != x.numel():
            raise ValueError("x and y must hold nsrc * 12V entries")
        rc = lib().sscg_apply_A_noalloc(self._h, _check_dev(x, "x"), _check_dev(y, "y"), nsrc, prec)
        if rc != OK:
            self._raise(rc)

    def shifted_cg_solve(self, v, z, sigma, y, opts: SolveOpts | None = None, true_res=True,
                         raise_on=(EINVAL, ENOMEM, EDEVICE, ESTATE)):
        nsrc = v.numel() // self.n
        z = np.asarray(z, dtype=np.complex128)
        N = z.size
        if y.numel() != nsrc * N * self.n:
            raise ValueError("y must hold nsrc * nshift * 12V entries")
        zz = _cplx_host(z)
        conv = np.zeros((nsrc, N), dtype=np.int32)
        tr = np.zeros((nsrc, N)) if true_res else None
        it = np.zeros(nsrc, dtype=np.int32)
        o = opts or default_opts()
        rc = lib().sscg_shifted_cg_solve(self._h, _check_dev(v, "v"), nsrc, _pd(zz), N, float(sigma),
                                         C.byref(o), _check_dev(y, "y"), _pi(conv),
                                         _pd(tr) if tr is not None else None, _pi(it))
        if rc in raise_on:
            self._raise(rc)
        return SolveResult(rc, conv, tr, it)

    def ss_moments(self, y, nshift, c, s):
        c = np.asarray(c, dtype=np.complex128)
        nmom = c.shape[0]
        nsrc = y.numel() // (nshift * self.n)
        cc = _cplx_host(c)
        rc = lib().sscg_ss_moments(self._h, _check_dev(y, "y"), nsrc, nshift, _pd(cc), nmom, _check_dev(s, "s"))
        if rc != OK:
            self._raise(rc)

    def ss_eigs(self, params: SSParams, v, max_eigs=64, want_vectors=True,
                raise_on=(EINVAL, ENOMEM, EDEVICE, ESTATE, EBREAKDOWN)):
        import torch
        nsrc = v.numel() // self.n
        lam = np.zeros(max(max_eigs, 1))
        res = np.zeros(max(max_eigs, 1))
        nf = np.zeros(1, dtype=np.int32)
        info = SSInfo()
        X = None
        if want_vectors and max_eigs > 0:
            X = torch.zeros((max_eigs, self.V, 4, 3), dtype=torch.complex128, device=v.device)
        rc = lib().sscg_ss_eigs(self._h, C.byref(params), _check_dev(v, "v"), nsrc, max_eigs, _pd(lam),
                                C.c_void_p(X.data_ptr()) if X is not None else None, _pd(res), _pi(nf),
                                C.byref(info))
        if rc in raise_on:
            self._raise(rc)
        k = min(int(nf[0]), max_eigs)
        return EigResult(rc, lam[:k].copy(), res[:k].copy(), int(nf[0]),
                         X[:k] if X is not None else None, info)

    def set_profiling(self, level=1):
        """0 off; 1 every launch timed (direct launches); k > 1 the dslash and shift
        update of every k-th iteration timed with graph replay kept on."""
        rc = lib().sscg_set_profiling(self._h, int(level))
        if rc:
            self._raise(rc)

    def stage_times(self):
        ms = np.zeros(8)
        calls = np.zeros(8, dtype=np.int64)
        lib().sscg_stage_times(self._h, _pd(ms), calls.ctypes.data_as(C.POINTER(C.c_int64)))
        return ms, calls

    def sweep_bytes(self):
        """Algorithmic HBM bytes of the block sweeps of the last solve (sscg_sweep_bytes)."""
        b = C.c_int64(0)
        rc = lib().sscg_sweep_bytes(self._h, C.byref(b))
        if rc:
            self._raise(rc)
        return int(b.value)

    def stage_launches(self):
        """Launches of each stage in the last solve (timed or not); index 6 = iterations."""
        n = np.zeros(8, dtype=np.int64)
        lib().sscg_stage_launches(self._h, n.ctypes.data_as(C.POINTER(C.c_int64)))
        return n


def batch_solve(ctxs, vs, zs, sigmas, ys, opts: SolveOpts | None = None, true_res=True):
    """Solve several problems (one per context) with grouped launches (sscg_batch_solve)."""
    P = len(ctxs)
    hs = (C.c_void_p * P)(*[c._h.value for c in ctxs])
    vp = (C.c_void_p * P)(*[_check_dev(v, "v").value for v in vs])
    yp = (C.c_void_p * P)(*[_check_dev(y, "y").value for y in ys])
    nsrc = np.array([v.numel() // c.n for c, v in zip(ctxs, vs)], dtype=np.int32)
    zz = [_cplx_host(z) for z in zs]
    nsh = np.array([z.size // 2 for z in zz], dtype=np.int32)
    zp = (C.POINTER(C.c_double) * P)(*[_pd(z) for z in zz])
    sg = np.asarray(sigmas, dtype=np.float64)
    conv = [np.zeros((int(nsrc[i]), int(nsh[i])), dtype=np.int32) for i in range(P)]
    tr = [np.zeros((int(nsrc[i]), int(nsh[i]))) for i in range(P)]
    it = [np.zeros(int(nsrc[i]), dtype=np.int32) for i in range(P)]
    cp = (C.POINTER(C.c_int32) * P)(*[_pi(a) for a in conv])
    tp = (C.POINTER(C.c_double) * P)(*[_pd(a) for a in tr])
    ip = (C.POINTER(C.c_int32) * P)(*[_pi(a) for a in it])
    o = opts or default_opts()
    rc = lib().sscg_batch_solve(hs, P, vp, _pi(nsrc), zp, _pi(nsh), _pd(sg), C.byref(o), yp, cp,
                                tp if true_res else None, ip)
    if rc in (EINVAL, ENOMEM, EDEVICE, ESTATE):
        raise SSCGError(rc, lib().sscg_last_error(ctxs[0]._h).decode())
    return [SolveResult(rc, conv[i], tr[i] if true_res else None, it[i]) for i in range(P)]
