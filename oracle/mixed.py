"""Mixed-precision Krylov with iterative refinement (not in the paper).

Outer loop in FP64: r = b - A x; stop when ||r||_2 <= rtol ||b||_2.
Inner solve of A e = r with the Krylov method of ``oracle.krylov`` carried
out in FP32 storage: matrix values and vectors rounded to float32, sparse
products accumulated in float32, inner products and norms accumulated in
float64.  The inner loop stops when its recursive residual drops below
inner_rtol * ||r||; then x += e in FP64.

Reading: inner tolerance 1e-4 by default, Jacobi preconditioner from the
FP32 diagonal, at most ``max_outer`` refinement steps (not converged after
that is reported as status 1).

``reliable_pcg`` is the variant used for the pressure solve: one Jacobi-PCG
whose recurrences run in FP32 while an FP64 accumulator holds the iterate;
whenever the FP32 recursive residual has dropped by a factor delta since
the last true residual (or below the tolerance), the FP32 correction is
added to the FP64 iterate, the true residual b - A x is recomputed in FP64
and replaces the recursive one, and the iteration continues with the same
search direction (residual replacement in the sense of van der Vorst and
Ye's reliable updates).  It stops when the FP64 true residual meets
rtol ||b||.  With FP64 recurrences it is plain Jacobi-PCG.
"""
from __future__ import annotations

import numpy as np

from .krylov import KrylovResult, NOTCONV, OK


def _pcg32(A32, d32, r, rtol, maxit):
    b = r.astype(np.float32)
    x = np.zeros_like(b)
    rr = b.copy()
    bn = float(np.sqrt(np.dot(b.astype(np.float64), b.astype(np.float64))))
    tol = rtol * bn
    z = (rr / d32).astype(np.float32)
    p = z.copy()
    rz = float(np.dot(rr.astype(np.float64), z.astype(np.float64)))
    it = 0
    while it < maxit:
        q = (A32 @ p).astype(np.float32)
        pq = float(np.dot(p.astype(np.float64), q.astype(np.float64)))
        if pq <= 0.0:
            break
        alpha = rz / pq
        x = (x + np.float32(alpha) * p).astype(np.float32)
        rr = (rr - np.float32(alpha) * q).astype(np.float32)
        it += 1
        if np.sqrt(np.dot(rr.astype(np.float64), rr.astype(np.float64))) <= tol:
            break
        z = (rr / d32).astype(np.float32)
        rz_new = float(np.dot(rr.astype(np.float64), z.astype(np.float64)))
        p = (z + np.float32(rz_new / rz) * p).astype(np.float32)
        rz = rz_new
    return x.astype(np.float64), it


def _bicgstab32(A32, d32, r0, rtol, maxit):
    """FP32 BiCGStab with right Jacobi preconditioning on A e = r0 (e0 = 0)."""
    f64 = lambda a: a.astype(np.float64)  # noqa: E731
    x = np.zeros(r0.size, dtype=np.float32)
    r = r0.astype(np.float32)
    tol = rtol * float(np.linalg.norm(r0))
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(r)
    p = np.zeros_like(r)
    it = 0
    while it < maxit:
        rho = float(np.dot(f64(rhat), f64(r)))
        if rho == 0.0:
            break
        beta = (rho / rho_old) * (alpha / omega)
        p = (r + np.float32(beta) * (p - np.float32(omega) * v)).astype(np.float32)
        ph = (p / d32).astype(np.float32)
        v = (A32 @ ph).astype(np.float32)
        rv = float(np.dot(f64(rhat), f64(v)))
        if rv == 0.0:
            break
        alpha = rho / rv
        s = (r - np.float32(alpha) * v).astype(np.float32)
        it += 1
        if np.linalg.norm(f64(s)) <= tol:
            x = (x + np.float32(alpha) * ph).astype(np.float32)
            break
        sh = (s / d32).astype(np.float32)
        t = (A32 @ sh).astype(np.float32)
        tt = float(np.dot(f64(t), f64(t)))
        omega = float(np.dot(f64(t), f64(s))) / tt if tt > 0 else 0.0
        x = (x + np.float32(alpha) * ph + np.float32(omega) * sh).astype(np.float32)
        r = (s - np.float32(omega) * t).astype(np.float32)
        if np.linalg.norm(f64(r)) <= tol or omega == 0.0:
            break
        rho_old = rho
    return x.astype(np.float64), it


def refine(method, A, b, x0, rtol=1e-8, inner_rtol=1e-4, maxit=10000, max_outer=50):
    """method: 'cg' or 'bicgstab'.  Returns KrylovResult with iters = total inner
    iterations and history = inner iterations per outer step."""
    A32 = A.astype(np.float32)
    d32 = A.diagonal().astype(np.float32)
    x = np.array(x0, dtype=np.float64, copy=True)
    bn = float(np.linalg.norm(b))
    total = 0
    hist = []
    inner = _pcg32 if method == "cg" else _bicgstab32
    for _ in range(max_outer):
        r = b - A @ x
        rn = float(np.linalg.norm(r))
        if rn <= rtol * bn:
            return KrylovResult(x, total, rn / bn, OK, hist)
        e, it = inner(A32, d32, r, inner_rtol, maxit - total)
        x += e
        total += it
        hist.append(it)
        if total >= maxit:
            break
    rn = float(np.linalg.norm(b - A @ x))
    return KrylovResult(x, total, rn / bn, OK if rn <= rtol * bn else NOTCONV, hist)


def reliable_pcg(A, b, x0, rtol=1e-8, delta=0.1, maxit=10000, inner_dtype=np.float32):
    """Reliable-update Jacobi-PCG (see the module docstring).  Returns
    KrylovResult with iters = CG iterations and history = the iteration
    numbers at which the residual was replaced."""
    lo = np.dtype(inner_dtype)
    f64 = lambda a: a.astype(np.float64)  # noqa: E731
    A_lo = A.astype(lo)
    d_lo = A.diagonal().astype(lo)
    x = np.array(x0, dtype=np.float64, copy=True)
    bn = float(np.linalg.norm(b))
    tol = rtol * bn
    r_hi = b - A @ x
    rn = float(np.linalg.norm(r_hi))
    if rn <= tol:
        return KrylovResult(x, 0, rn / bn if bn > 0 else rn, OK, [])
    r = r_hi.astype(lo)
    x_lo = np.zeros_like(r)
    upd = delta * rn
    z = (r / d_lo).astype(lo)
    rz = float(np.dot(f64(r), f64(z)))
    p = z.copy()
    it = 0
    replaced = []
    while it < maxit:
        q = (A_lo @ p).astype(lo)
        pq = float(np.dot(f64(p), f64(q)))
        if not pq > 0.0:
            break
        alpha = lo.type(rz / pq)
        x_lo = (x_lo + alpha * p).astype(lo)
        r = (r - alpha * q).astype(lo)
        it += 1
        rn_lo = float(np.sqrt(np.dot(f64(r), f64(r))))
        if rn_lo <= tol or rn_lo <= upd:
            x += f64(x_lo)
            r_hi = b - A @ x
            rn = float(np.linalg.norm(r_hi))
            replaced.append(it)
            if rn <= tol:
                return KrylovResult(x, it, rn / bn, OK, replaced)
            r = r_hi.astype(lo)
            x_lo = np.zeros_like(r)
            upd = delta * rn
        z = (r / d_lo).astype(lo)
        rz_new = float(np.dot(f64(r), f64(z)))
        p = (z + lo.type(rz_new / rz) * p).astype(lo)
        rz = rz_new
    x += f64(x_lo)
    rn = float(np.linalg.norm(b - A @ x))
    return KrylovResult(x, it, rn / bn, OK if rn <= tol else NOTCONV, replaced)
