"""Textbook Krylov solvers with Jacobi preconditioning (FP64).

The paper solves the tentative-velocity systems with BiCGStab + Jacobi and
the pressure correction with a symmetric Krylov method (Sec. 6.2, channel
performance paragraph); the pressure solver here is Jacobi-preconditioned CG.

Readings taken where the paper is silent:
* Stopping test on the true residual: ||b - A x||_2 <= rtol * ||b||_2,
  atol = 0.  The recursively updated residual triggers the test, which is
  then confirmed with an explicit b - A x; if that fails the loop continues
  from the explicit residual.
* BiCGStab uses right Jacobi preconditioning (the operator A D^{-1}, with D
  the diagonal of A after Dirichlet rows have been replaced by identity
  rows), shadow residual r_hat = r_0, and the early exit on ||s||.  On a
  breakdown (rho = 0, (r_hat, v) = 0 or omega = 0) it restarts once with
  r_hat = r, and a second breakdown is reported.
* Status codes: 0 converged, 1 not converged within maxit, 2 breakdown,
  3 non-finite values.
"""
from __future__ import annotations

import dataclasses

import numpy as np

OK, NOTCONV, BREAKDOWN, NAN = 0, 1, 2, 3


@dataclasses.dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    rel_res: float        # true ||b - A x|| / ||b||
    status: int
    history: list


def _true_rel(A, b, x, bnorm):
    return float(np.linalg.norm(b - A @ x) / bnorm) if bnorm > 0 else float(np.linalg.norm(b - A @ x))


def pcg(A, b, x0, rtol=1e-8, maxit=10000, diag=None, history=False):
    """Jacobi-preconditioned conjugate gradients (Hestenes-Stiefel)."""
    d = A.diagonal() if diag is None else diag
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    tol = rtol * bnorm
    r = b - A @ x
    hist = [float(np.linalg.norm(r))] if history else []
    if not np.all(np.isfinite(r)):
        return KrylovResult(x, 0, float("nan"), NAN, hist)
    if np.linalg.norm(r) <= tol:
        return KrylovResult(x, 0, _true_rel(A, b, x, bnorm), OK, hist)
    z = r / d
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit:
        q = A @ p
        pq = float(p @ q)
        if not np.isfinite(pq):
            return KrylovResult(x, it, float("nan"), NAN, hist)
        if pq <= 0.0:
            return KrylovResult(x, it, _true_rel(A, b, x, bnorm), BREAKDOWN, hist)
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        if history:
            hist.append(rn)
        if not np.isfinite(rn):
            return KrylovResult(x, it, float("nan"), NAN, hist)
        if rn <= tol:
            r_true = b - A @ x
            if np.linalg.norm(r_true) <= tol:
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), OK, hist)
            r = r_true                       # continue from the explicit residual
            z = r / d
            p = z.copy()
            rz = float(r @ z)
            continue
        z = r / d
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return KrylovResult(x, it, _true_rel(A, b, x, bnorm), NOTCONV, hist)


def bicgstab(A, b, x0, rtol=1e-8, maxit=10000, diag=None, history=False):
    """BiCGStab (van der Vorst) with right Jacobi preconditioning: the
    iteration runs on A D^{-1} y = b with x = D^{-1} y, written in x so that
    p_hat = D^{-1} p and s_hat = D^{-1} s are the preconditioned directions.
    Its residual r is the true residual b - A x."""
    d = A.diagonal() if diag is None else diag
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    tol = rtol * bnorm
    r = b - A @ x
    hist = [float(np.linalg.norm(r))] if history else []
    if not np.all(np.isfinite(r)):
        return KrylovResult(x, 0, float("nan"), NAN, hist)
    if np.linalg.norm(r) <= tol:
        return KrylovResult(x, 0, _true_rel(A, b, x, bnorm), OK, hist)
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(x)
    p = np.zeros_like(x)
    restarted = False
    it = 0

    def restart():
        return r.copy(), 1.0, 1.0, 1.0, np.zeros_like(x), np.zeros_like(x)

    while it < maxit:
        rho = float(rhat @ r)
        if rho == 0.0:
            if restarted:
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), BREAKDOWN, hist)
            restarted = True
            rhat, rho_old, alpha, omega, v, p = restart()
            continue
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = p / d
        v = A @ ph
        rv = float(rhat @ v)
        if rv == 0.0 or not np.isfinite(rv):
            if not np.isfinite(rv):
                return KrylovResult(x, it, float("nan"), NAN, hist)
            if restarted:
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), BREAKDOWN, hist)
            restarted = True
            rhat, rho_old, alpha, omega, v, p = restart()
            continue
        alpha = rho / rv
        s = r - alpha * v
        it += 1
        sn = float(np.linalg.norm(s))
        if sn <= tol:
            xs = x + alpha * ph
            if np.linalg.norm(b - A @ xs) <= tol:
                x = xs
                if history:
                    hist.append(sn)
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), OK, hist)
        sh = s / d
        t = A @ sh
        tt = float(t @ t)
        omega = float(t @ s) / tt if tt > 0.0 else 0.0
        x += alpha * ph + omega * sh
        r = s - omega * t
        rn = float(np.linalg.norm(r))
        if history:
            hist.append(rn)
        if not np.isfinite(rn):
            return KrylovResult(x, it, float("nan"), NAN, hist)
        if rn <= tol:
            r_true = b - A @ x
            if np.linalg.norm(r_true) <= tol:
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), OK, hist)
            r = r_true
        if omega == 0.0:
            if restarted:
                return KrylovResult(x, it, _true_rel(A, b, x, bnorm), BREAKDOWN, hist)
            restarted = True
            rhat, rho_old, alpha, omega, v, p = restart()
            continue
        rho_old = rho
    return KrylovResult(x, it, _true_rel(A, b, x, bnorm), NOTCONV, hist)
