"""Krylov solvers in plain NumPy FP64 (oracle; test infrastructure only).

* ``gcr``      flexible generalized conjugate residuals with restarts; the
               outer solver of the paper (adaptive multigrid paragraph) and
               the per-level solver of the recursive cycle (Implementation
               paragraph).  The preconditioner may change between calls.
* ``bicgstab`` van der Vorst's BiCGStab, the conventional Krylov solver of
               the Introduction, run in plain FP64.
* ``mr``       minimal-residual relaxation, used as the smoother (the paper
               leaves the smoother type open; MR is the reading used).

All vectors are NumPy arrays of any shape; inner products are np.vdot.
"""
import numpy as np


def norm(v):
    return float(np.sqrt(np.vdot(v, v).real))


class SolveInfo:
    def __init__(self):
        self.iters = 0
        self.history = []
        self.converged = False
        self.restarts = 0


def gcr(A, b, x0=None, tol=1e-10, restart=16, maxiter=1000, precond=None,
        target_norm=None, info=None):
    """Flexible GCR.  Stops when ||b - A x|| <= tol * target_norm.

    target_norm defaults to ||b||.  The residual is recomputed from scratch
    at every restart.  Returns x (and fills `info` when given).
    """
    info = info if info is not None else SolveInfo()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    r = b - A(x) if x0 is not None else b.copy()
    target = tol * (norm(b) if target_norm is None else target_norm)
    rn = norm(r)
    info.history.append(rn)
    if rn <= target:
        info.converged = True
        return x
    while info.iters < maxiter:
        Z, Q = [], []
        for _ in range(restart):
            z = precond(r) if precond is not None else r.copy()
            q = A(z)
            for zi, qi in zip(Z, Q):
                beta = np.vdot(qi, q)
                q = q - beta * qi
                z = z - beta * zi
            nq = norm(q)
            if nq == 0.0:
                break
            q = q / nq
            z = z / nq
            alpha = np.vdot(q, r)
            x = x + alpha * z
            r = r - alpha * q
            Z.append(z)
            Q.append(q)
            info.iters += 1
            rn = norm(r)
            info.history.append(rn)
            if rn <= target or info.iters >= maxiter:
                break
        r = b - A(x)
        rn = norm(r)
        info.restarts += 1
        if rn <= target:
            info.converged = True
            break
    return x


def bicgstab(A, b, x0=None, tol=1e-10, maxiter=10000, target_norm=None, info=None):
    """Plain BiCGStab; stop when ||r|| <= tol * target_norm (default ||b||)."""
    info = info if info is not None else SolveInfo()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    r = b - A(x) if x0 is not None else b.copy()
    target = tol * (norm(b) if target_norm is None else target_norm)
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    rn = norm(r)
    info.history.append(rn)
    while rn > target and info.iters < maxiter:
        rho_new = np.vdot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho_new / np.vdot(rhat, v)
        s = r - alpha * v
        t = A(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        info.iters += 1
        rn = norm(r)
        info.history.append(rn)
    info.converged = rn <= target
    return x


def mr(A, b, x0, iters):
    """`iters` steps of minimal-residual relaxation on A x = b from x0."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = b - A(x)
    for _ in range(iters):
        Ar = A(r)
        den = np.vdot(Ar, Ar).real
        if den == 0.0:
            break
        a = np.vdot(Ar, r) / den
        x = x + a * r
        r = r - a * Ar
    return x
