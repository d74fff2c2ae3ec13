"""The dense DDA system (paper Sec. 2.1-2.2).  Test infrastructure only.

Vector layouts
--------------
* box:     complex128 [3][nz][ny][nx] — every voxel of the bounding box; air
           entries of the solution are zero.
* compact: complex128 [3 * n_occ] — occupied voxels only, component-major
           (all x-components in C order of the grid, then y, then z).

The system matrix on the compact unknowns is (Sec. 2.2, the 3x3 block display)
    A = diag(alpha^{-1}) - d^3 G,
with G_ab(r_i - r_j) between distinct occupied voxels and nothing on the
diagonal (midpoint rule, eq. midpoint; self term by eq. CM).
"""

from __future__ import annotations

import numpy as np

from .physics import alpha_inv, green, lattice_S


def centres(shape, d: float):
    """Voxel centre coordinates, grid centred on the origin: array [nz][ny][nx][3] (x, y, z)."""
    nz, ny, nx = shape
    x = (np.arange(nx) - (nx - 1) / 2.0) * d
    y = (np.arange(ny) - (ny - 1) / 2.0) * d
    z = (np.arange(nz) - (nz - 1) / 2.0) * d
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def incident_field(mask, k: float, d: float, direction, polarisation):
    """E^inc at voxel centres (box layout, zero in air): pol * exp(i k dir . r)."""
    r = centres(mask.shape, d)
    phase = np.exp(1j * k * (r @ np.asarray(direction, dtype=np.float64)))
    pol = np.asarray(polarisation, dtype=np.float64)
    b = pol[:, None, None, None] * phase[None]
    return b * mask[None].astype(np.float64)


def alpha_inv_box(mask, eps, k: float, d: float, direction, polarisation):
    """Per-voxel alpha^{-1} (box layout, meaningless in air) for one incident wave."""
    S = lattice_S(direction, polarisation)
    return alpha_inv(eps, k * d, S)


def box_to_compact(xbox, mask):
    occ = mask.astype(bool).ravel()
    return np.concatenate([xbox[a].ravel()[occ] for a in range(3)])


def compact_to_box(xc, mask):
    occ = mask.astype(bool).ravel()
    n = int(occ.sum())
    out = np.zeros((3,) + mask.shape, dtype=np.complex128)
    for a in range(3):
        out[a].reshape(-1)[occ] = xc[a * n:(a + 1) * n]
    return out


def dense_matrix(mask, eps, k: float, d: float, S: float):
    """The full 3 n_occ x 3 n_occ DDA matrix on the occupied voxels (compact order)."""
    occ = mask.astype(bool).ravel()
    r = centres(mask.shape, d).reshape(-1, 3)[occ]
    n = r.shape[0]
    G = green(r[:, None, :] - r[None, :, :], k)  # [n][n][3][3], zero on the diagonal
    A = np.empty((3 * n, 3 * n), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            A[a * n:(a + 1) * n, b * n:(b + 1) * n] = -(d ** 3) * G[:, :, a, b]
    ainv = alpha_inv(eps.ravel()[occ], k * d, S)
    idx = np.arange(3 * n)
    A[idx, idx] += np.tile(ainv, 3)
    return A


def box_operator_dense(mask, eps, k, d, S, xbox):
    """Full-box operator built from the dense matrix: y = M (A x) on occupied, x in air."""
    A = dense_matrix(mask, eps, k, d, S)
    yc = A @ box_to_compact(xbox, mask)
    y = compact_to_box(yc, mask)
    air = ~mask.astype(bool)
    y[:, air] = xbox[:, air]
    return y
