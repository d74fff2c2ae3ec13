"""BiCGStab, right-preconditioned (paper Sec. 4: the second solver, tolerance 1e-5, cap 4000).

Test infrastructure only.  The stabilised biconjugate-gradient method of van der Vorst
(1992) for complex systems, with conjugated inner products a^H b, applied to A P^{-1} u = b
and x = P^{-1} u, x0 = 0 unless given.  One iteration is one pass through the recurrence
(two operator and two preconditioner applications).  Stopping: the updated residual
||r|| / ||b|| <= tol after an iteration; the true residual ||b - A x|| / ||b|| is then formed,
and if it is above tol (the updated residual drifts in finite precision) the method restarts
from it.  A zero denominator (breakdown) also restarts from the true residual, once per
occurrence, within the iteration cap.
"""

from __future__ import annotations

import numpy as np


def bicgstab(matvec, b, precond=None, tol: float = 1e-5, maxit: int = 4000, x0=None):
    """Solve A x = b.  ``matvec`` and ``precond`` (v -> P^{-1} v) act on arrays of b's shape.

    Returns (x, info) with info = dict(converged, iters, restarts, rel_residual, history)
    where history is the updated residual / ||b|| after each iteration.
    """
    if precond is None:
        def precond(v):
            return v
    shape = b.shape
    bv = b.ravel()
    bnorm = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    info = dict(converged=False, iters=0, restarts=0, rel_residual=np.inf, history=[])
    if bnorm == 0.0:
        info.update(converged=True, rel_residual=0.0)
        return x.reshape(shape), info

    def A(v):
        return matvec(v.reshape(shape)).ravel()

    def M(v):
        return precond(v.reshape(shape)).ravel()

    iters = 0
    while True:
        r = bv - A(x)
        rel = np.linalg.norm(r) / bnorm
        info["rel_residual"] = rel
        if rel <= tol:
            info["converged"] = True
            break
        if iters >= maxit:
            break
        rhat = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(bv)
        p = np.zeros_like(bv)
        restart = False
        start = iters
        while iters < maxit:
            rho_new = np.vdot(rhat, r)
            if rho_new == 0.0:
                restart = True
                break
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = M(p)
            v = A(ph)
            den = np.vdot(rhat, v)
            if den == 0.0:
                restart = True
                break
            alpha = rho_new / den
            s = r - alpha * v
            sh = M(s)
            t = A(sh)
            tt = np.vdot(t, t)
            if tt == 0.0:  # s = 0 up to t: the half step already solves the system
                x = x + alpha * ph
                iters += 1
                break
            omega = np.vdot(t, s) / tt
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            iters += 1
            rho = rho_new
            info["history"].append(np.linalg.norm(r) / bnorm)
            if info["history"][-1] <= tol or omega == 0.0:
                break
        info["restarts"] += 1
        if restart and iters == start:  # breakdown before any progress: give up
            info["rel_residual"] = np.linalg.norm(bv - A(x)) / bnorm
            break
        if not restart and iters >= maxit:
            r = bv - A(x)
            info["rel_residual"] = np.linalg.norm(r) / bnorm
            info["converged"] = info["rel_residual"] <= tol
            break
    info["iters"] = iters
    info["restarts"] = max(0, info["restarts"] - 1)
    return x.reshape(shape), info
