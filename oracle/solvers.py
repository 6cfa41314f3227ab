"""Shifted linear systems (z_j I - A) y_j = v, eq. (4) (oracle; test infrastructure only).

Two independent routes:
  normal_cg       textbook CG, one run per shift, on the Hermitian positive definite
                  normal equations (z_j I - A)^H (z_j I - A) y = (z_j I - A)^H v: a
                  route to each y_j that shares nothing with the shifted recurrences
                  (used to certify the stored solutions of the 8^4 workload).
  shifted_cg      the method of Sec. 2.2: CG on the Hermitian seed system
                  (sigma I - A) x = v with a real seed shift sigma, whose residuals
                  give the residuals of every shifted system by collinearity
                  (r^s_k = xi^s_k r_k, eq. 5 and the text after it). Because the
                  seed matrix is Hermitian, the shadow residual of BiCG equals the
                  residual and one matrix-vector product per iteration serves all
                  shifts.
"""
from __future__ import annotations

import numpy as np


def normal_cg(A_mul, z: np.ndarray, V: np.ndarray, tol: float = 1e-13, maxiter: int = 100000):
    """Per-shift solves by CG on the normal equations, all columns at once.

    A_mul(X) applies A to a block of vectors X [m][n]. V is [m][n] (one source per
    shift, broadcast by the caller). With B_j = z_j I - A, CG runs on
    B_j^H B_j y = B_j^H v_j, which is Hermitian positive definite because A is
    Hermitian and Im z_j != 0 or z_j is not an eigenvalue. Stops when every true
    relative residual ||v - B_j y_j|| / ||v|| is below tol.
    """
    z = np.asarray(z)[:, None]
    Bmul = lambda X: z * X - A_mul(X)
    BHmul = lambda X: np.conj(z) * X - A_mul(X)
    vn = np.linalg.norm(V, axis=1)
    Y = np.zeros_like(V)
    r = BHmul(V)
    p = r.copy()
    rr = np.einsum("ij,ij->i", r.conj(), r).real
    for it in range(maxiter):
        q = BHmul(Bmul(p))
        a = rr / np.einsum("ij,ij->i", p.conj(), q).real
        Y += a[:, None] * p
        r -= a[:, None] * q
        rr_new = np.einsum("ij,ij->i", r.conj(), r).real
        if it % 20 == 0 or it == maxiter - 1:
            res = np.linalg.norm(V - Bmul(Y), axis=1) / vn
            if np.all(res < tol):
                break
        p = r + (rr_new / rr)[:, None] * p
        rr = rr_new
    return Y


class ShiftedCGResult:
    def __init__(self, Y, conv_iter, iters, status, history=None):
        self.Y = Y                  # [N][n] shifted solutions
        self.conv_iter = conv_iter  # [N] iteration after which each shift froze, -1 if never
        self.iters = iters          # seed iterations performed
        self.status = status        # "ok", "notconv", "breakdown"
        self.history = history


def shifted_cg(A_mul, v: np.ndarray, z: np.ndarray, sigma: float, tol: float = 1e-12,
               maxiter: int = 100000, record=None, tol_scale=None, fp32_switch=None, fold_every=50):
    """Shifted CG with a real Hermitian seed (Sec. 2.2).

    Seed matrix B = sigma I - A (Hermitian because sigma is real); shift j is
    z_j I - A = B + s_j I with s_j = z_j - sigma. The seed runs plain CG:
        q = B p_k,  alpha_k = rho_k / <p_k, q>,  r_{k+1} = r_k - alpha_k q,
        beta_k = rho_{k+1} / rho_k,  p_{k+1} = r_{k+1} + beta_k p_k.
    The seed residual is R_k(B) v with R_k the CG residual polynomial, which obeys
        R_{k+1}(t) = (1 - alpha_k t + alpha_k beta_{k-1}/alpha_{k-1}) R_k(t)
                     - (alpha_k beta_{k-1}/alpha_{k-1}) R_{k-1}(t).
    Shift j lives in the same Krylov space, so its residual is collinear with the
    seed's: r^j_k = r_k / pi_{j,k} with pi_{j,k} = R_k(-s_j) (the xi of eq. 5 is
    1/pi). Hence
        pi_{j,k+1} = (1 + alpha_k beta_{k-1}/alpha_{k-1} + alpha_k s_j) pi_{j,k}
                     - (alpha_k beta_{k-1}/alpha_{k-1}) pi_{j,k-1},
        alpha_{j,k} = alpha_k pi_{j,k}/pi_{j,k+1},
        beta_{j,k}  = (pi_{j,k}/pi_{j,k+1})^2 beta_k,
        x_j += alpha_{j,k} p_j,   p_j <- r_{k+1}/pi_{j,k+1} + beta_{j,k} p_j,
    starting from x_j = 0, p_j = v, pi_{j,-1} = pi_{j,0} = 1, alpha_{-1} = 1,
    beta_{-1} = 0.
    Stopping rule (reading of Sec. 4's criterion, applied per shift): after its update
    in iteration k, shift j freezes once sqrt(rho_{k+1}) / |pi_{j,k+1}| <= tol ||v||;
    conv_iter[j] = k + 1. The run ends when every shift has frozen. tol_scale (one
    factor per shift) replaces tol by tol * tol_scale[j] for shift j.

    fp32_switch (precision emulation, not in the paper): once every active shift's
    relative residual sqrt(rho)/|pi_j|/||v|| is below fp32_switch, the shift vectors
    p_j are held in complex64 and updated in complex64 arithmetic (with the FP64
    scalars rounded to complex64), their steps alpha_j p_j are summed into a complex64
    partial solution, and that partial is added to the FP64 solution every fold_every
    iterations and at the end. The seed stays FP64. This is the precision schedule
    whose errors the FP32-shift mode of the GPU path has to stay within.

    A_mul(x) applies A to one vector. record(k, state) is called after every
    iteration when given (used to compare iterates at a fixed k).
    """
    v = np.asarray(v, dtype=np.complex128)
    z = np.asarray(z, dtype=np.complex128)
    N = z.size
    s = z - sigma
    vnorm = np.linalg.norm(v)
    if vnorm == 0 or not np.isfinite(vnorm):
        raise ValueError("source must be nonzero and finite")
    r = v.copy()
    p = v.copy()
    rho = np.vdot(r, r).real
    X = np.zeros((N, v.size), dtype=np.complex128)
    P = np.tile(v, (N, 1))
    pi_prev = np.ones(N, dtype=np.complex128)
    pi_cur = np.ones(N, dtype=np.complex128)
    alpha_prev, beta_prev = 1.0, 0.0
    active = np.ones(N, dtype=bool)
    conv_iter = np.full(N, -1, dtype=np.int64)
    P32 = None           # complex64 shift vectors once switched
    X32 = None           # complex64 partial solutions
    since = 0            # iterations since the last fold
    thr = tol * vnorm * (np.ones(N) if tol_scale is None else np.asarray(tol_scale, dtype=np.float64))
    status = "notconv"
    k = 0
    for k in range(maxiter):
        q = sigma * p - A_mul(p)
        pq = np.vdot(p, q).real
        if pq == 0 or not np.isfinite(pq):
            status = "breakdown"
            break
        alpha = rho / pq
        c = alpha * beta_prev / alpha_prev
        pi_next = (1 + c + alpha * s) * pi_cur - c * pi_prev
        r = r - alpha * q
        rho_next = np.vdot(r, r).real
        beta = rho_next / rho
        ratio = pi_cur / pi_next
        a_j = alpha * ratio
        b_j = ratio ** 2 * beta
        act = np.nonzero(active)[0]
        if P32 is None:
            X[act] += a_j[act, None] * P[act]
            P[act] = r[None, :] / pi_next[act, None] + b_j[act, None] * P[act]
        else:
            a32 = a_j.astype(np.complex64)
            b32 = b_j.astype(np.complex64)
            ipi32 = (1.0 / pi_next).astype(np.complex64)
            r32 = r.astype(np.complex64)
            X32[act] += a32[act, None] * P32[act]
            P32[act] = ipi32[act, None] * r32[None, :] + b32[act, None] * P32[act]
            since += 1
            if since == fold_every:
                X += X32.astype(np.complex128)
                X32[:] = 0
                since = 0
        p = r + beta * p
        newly = active & (np.sqrt(rho_next) / np.abs(pi_next) <= thr)
        conv_iter[newly] = k + 1
        active &= ~newly
        pi_prev, pi_cur = pi_cur, pi_next
        alpha_prev, beta_prev, rho = alpha, beta, rho_next
        if (fp32_switch is not None and P32 is None and active.any()
                and np.max(np.sqrt(rho) / np.abs(pi_cur[active])) / vnorm < fp32_switch):
            P32 = P.astype(np.complex64)
            X32 = np.zeros_like(P32)
        if record is not None:
            record(k, dict(X=X, P=P, r=r, p=p, pi=pi_cur, alpha=alpha, beta=beta, rho=rho,
                           updated=act.size, active=active))
        if not active.any():
            status = "ok"
            k += 1
            break
        if not np.isfinite(rho) or rho == 0:
            status = "breakdown"
            k += 1
            break
    else:
        k = maxiter
    if X32 is not None:
        X += X32.astype(np.complex128)
    return ShiftedCGResult(X, conv_iter, k, status)


def true_residuals(A_mul, v, z, Y):
    """||v - (z_j I - A) y_j|| / ||v|| for every shift."""
    vn = np.linalg.norm(v)
    return np.array([np.linalg.norm(v - (zj * y - A_mul(y))) / vn for zj, y in zip(z, Y)])
