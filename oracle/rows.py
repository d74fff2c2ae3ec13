"""Sampled rows by direct summation, for grids too large to assemble anything.

Test infrastructure only.  Each function evaluates a few output entries of an
operator straight from its definition, one voxel at a time, in O(N) work per
sampled voxel — the check used at full benchmark sizes.
"""

from __future__ import annotations

import numpy as np

from .circulant import FULL, two_level_generator
from .physics import alpha_inv, green
from .system import centres


def operator_rows(samples, xbox, mask, eps, k, d, S):
    """y_i = alpha_i^{-1} x_i - sum_{j != i, occupied} d^3 G(r_i - r_j) x_j for sampled
    occupied voxels i (flat C-order indices).  Returns [len(samples)][3]."""
    occ = mask.astype(bool).ravel()
    r = centres(mask.shape, d).reshape(-1, 3)
    rj = r[occ]
    xj = np.stack([xbox[a].ravel()[occ] for a in range(3)], axis=-1)  # [n][3]
    eflat = eps.ravel()
    out = np.empty((len(samples), 3), dtype=np.complex128)
    for t, i in enumerate(samples):
        G = green(r[i][None, :] - rj, k)  # zero where j == i
        conv = d ** 3 * np.einsum("jab,jb->a", G, xj)
        ai = alpha_inv(eflat[i], k * d, S)
        xi = np.array([xbox[a].ravel()[i] for a in range(3)])
        out[t] = ai * xi - conv
    return out


def precond_rows(samples, zbox, k, d, alpha_tilde_inv, generator=None):
    """(P z)_i for P = alpha~^{-1} I - C2 on a fully occupied box, where C2 is the
    2-level circulant (x, y) / Toeplitz (z) matrix of the eq. Chan generator.
    Returns [len(samples)][3]."""
    _, nz, ny, nx = zbox.shape
    c2 = two_level_generator((nz, ny, nx), k, d) if generator is None else generator
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty((len(samples), 3), dtype=np.complex128)
    for t, i in enumerate(samples):
        sz, sy, sx = np.unravel_index(i, (nz, ny, nx))
        ds = (sz - iz) + nz - 1
        dq = (sy - iy) % ny
        dp = (sx - ix) % nx
        row = np.zeros(3, dtype=np.complex128)
        for a in range(3):
            acc = 0.0 + 0.0j
            for b in range(3):
                acc += np.sum(c2[FULL[a, b]][ds, dq, dp] * zbox[b])
            row[a] = alpha_tilde_inv * zbox[a, sz, sy, sx] - acc
        out[t] = row
    return out
