"""Adjoint gradient of the extinction cross section w.r.t. per-voxel permittivity.

Test infrastructure only.  Not in the paper; derived from its system (Sec. 2.1-2.2):
with h = E_inc^H c and A c = E_inc, dh = -lambda^T (dA) c where A lambda = conj(E_inc)
(A is complex symmetric, so A^T = A).  dA is diagonal: d(alpha_j^{-1})/d eps_j on
the three components of voxel j.  C_ext = 4 pi k d^3 Im h and h is holomorphic in
eps, so with h'_j = -(d alpha_j^{-1}/d eps_j) sum_a lambda_{j,a} c_{j,a}:
    dC/d Re eps_j = 4 pi k d^3 Im h'_j,   dC/d Im eps_j = 4 pi k d^3 Re h'_j,
and the complex gradient (dC/dRe + i dC/dIm) is 4 pi k d^3 * i * conj(h'_j).
"""

from __future__ import annotations

import numpy as np

from .physics import dalpha_inv_deps, lattice_S
from .system import box_to_compact, compact_to_box, dense_matrix, incident_field


def gradient_from_fields(cbox, lbox, mask, eps, k, d, direction, polarisation):
    """Complex gradient [nz][ny][nx] (zero in air) from forward and adjoint solutions."""
    S = lattice_S(direction, polarisation)
    occ = mask.astype(bool)
    dai = np.where(occ, dalpha_inv_deps(np.where(occ, eps, 2.0), k * d, S), 0.0)
    hp = -dai * np.sum(lbox * cbox, axis=0)
    g = 4.0 * np.pi * k * d ** 3 * 1j * np.conj(hp)
    return g * mask


def grad_cext_dense(mask, eps, k, d, direction, polarisation):
    """(C_ext, gradient) with both solves by dense LU (small grids)."""
    S = lattice_S(direction, polarisation)
    A = dense_matrix(mask, eps, k, d, S)
    b = incident_field(mask, k, d, direction, polarisation)
    bc = box_to_compact(b, mask)
    c = np.linalg.solve(A, bc)
    lam = np.linalg.solve(A, np.conj(bc))
    cbox, lbox = compact_to_box(c, mask), compact_to_box(lam, mask)
    cext = float(4.0 * np.pi * k * d ** 3 * np.imag(np.vdot(bc, c)))
    return cext, gradient_from_fields(cbox, lbox, mask, eps, k, d, direction, polarisation)
