"""Restarted GMRES, right- or left-preconditioned (paper Sec. 4 uses GMRES to tolerance 1e-5).

Test infrastructure only.  Modified Gram-Schmidt Arnoldi with Givens rotations
(the textbook form of Saad & Schultz), x0 = 0 unless given.  The paper keeps
the full Krylov space; restarts every ``restart`` iterations are used here (the
paper recommends trying restarts, Sec. 4-5).  Right preconditioning (the
default): the Givens estimate of the residual of A P^{-1} u = b is checked after
every iteration; at the end of each cycle the true residual ||b - A x|| / ||b||
decides convergence.  Left preconditioning, the paper's eq. (general_prec),
P^{-1} A x = P^{-1} b: plain GMRES on that system, so every test is on
||P^{-1} (b - A x)|| / ||P^{-1} b||.
"""

from __future__ import annotations

import numpy as np


def gmres(matvec, b, precond=None, restart: int = 30, tol: float = 1e-5, maxit: int = 2000,
          x0=None, side: str = "right"):
    """Solve A x = b.  ``matvec`` and ``precond`` (x -> P^{-1} x) act on arrays of b's shape.

    Returns (x, info) with info = dict(converged, iters, cycles, rel_residual,
    history) where history is the per-iteration Givens estimate / ||b||.  With
    side="left" the system solved is P^{-1} A x = P^{-1} b: rel_residual and history
    are those of that system, and info["true_rel_residual"] is ||b - A x|| / ||b||.
    """
    if side == "left" and precond is not None:
        pb = precond(b)
        x, info = gmres(lambda v: precond(matvec(v)), pb, None, restart, tol, maxit, x0)
        r = b.ravel() - matvec(x).ravel()
        bn = np.linalg.norm(b.ravel())
        info["true_rel_residual"] = np.linalg.norm(r) / bn if bn > 0 else 0.0
        return x, info
    if side not in ("left", "right"):
        raise ValueError(f"side must be 'left' or 'right', got {side!r}")
    if precond is None:
        def precond(v):
            return v
    shape = b.shape
    bv = b.ravel()
    bnorm = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    info = dict(converged=False, iters=0, cycles=0, rel_residual=np.inf, history=[])
    if bnorm == 0.0:
        info.update(converged=True, rel_residual=0.0)
        return x.reshape(shape), info
    r = bv - matvec(x.reshape(shape)).ravel()
    beta = np.linalg.norm(r)
    info["rel_residual"] = beta / bnorm
    if beta / bnorm <= tol:
        info["converged"] = True
        return x.reshape(shape), info
    iters = 0
    while iters < maxit:
        info["cycles"] += 1
        V = np.zeros((restart + 1, bv.size), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        j_used = 0
        for j in range(restart):
            w = matvec(precond(V[j].reshape(shape)).reshape(shape)).ravel()
            iters += 1
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            elif abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            info["history"].append(abs(g[j + 1]) / bnorm)
            j_used = j + 1
            if abs(g[j + 1]) / bnorm <= tol or iters >= maxit or breakdown:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        u = V[:j_used].T @ y
        x = x + precond(u.reshape(shape)).ravel()
        r = bv - matvec(x.reshape(shape)).ravel()
        beta = np.linalg.norm(r)
        info["rel_residual"] = beta / bnorm
        if beta / bnorm <= tol:
            info["converged"] = True
            break
    info["iters"] = iters
    return x.reshape(shape), info
