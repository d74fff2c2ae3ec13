"""T. Chan's optimal circulant and the 2-level block preconditioner (paper Sec. 3).

Test infrastructure only.

Two independent routes are provided so that each pins the other:

* brute force (``two_level_dense``): build the full-box BTTB matrix d^3 G over
  all 3N box unknowns, replace every l x l Toeplitz block along x by the
  Frobenius-nearest circulant (average of each wrapped diagonal — the property
  eq. Chan is derived from), then do the same along y; P = alpha~^{-1} I - C2
  (Sec. 3.1, the definition of C_B2 with the constant diagonal).
* formula (``two_level_blocks``): eq. Chan applied to the signed-offset kernel
  along x then along y, a 2-D DFT over the two circulant levels, and for each
  of the l*m Fourier modes the dense 3n x 3n block (Toeplitz along z) that the
  permutation of Sec. 3 exposes; this is Algorithms 2-3 of Sec. 3.1 applied to
  all six components with their parities handled implicitly by using signed
  offsets (no first-row / first-column sign bookkeeping).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fftmatvec import kernel_signed
from .physics import COMP6

FULL = np.zeros((3, 3), dtype=int)
for _c, (_a, _b) in enumerate(COMP6):
    FULL[_a, _b] = FULL[_b, _a] = _c


def chan_column(t_signed):
    """Eq. Chan: first column of T. Chan's circulant from Toeplitz t_p, p in (-l, l).

    ``t_signed[..., p + l - 1] = t_p`` along the last axis; returns
    c_p = ((l - p) t_p + p t_{p - l}) / l for p = 0 .. l-1 (last axis).
    """
    L2 = t_signed.shape[-1]
    l = (L2 + 1) // 2
    p = np.arange(l)
    pos = t_signed[..., l - 1 + p]
    neg = np.zeros_like(pos)
    neg[..., 1:] = t_signed[..., p[1:] - 1]  # t_{p - l} sits at index p - 1
    return ((l - p) * pos + p * neg) / l


def toeplitz_from_signed(t_signed):
    """Dense Toeplitz T[i, j] = t_{i-j} from t_p, p in (-l, l)."""
    L2 = t_signed.shape[-1]
    l = (L2 + 1) // 2
    i = np.arange(l)
    return t_signed[(i[:, None] - i[None, :]) + l - 1]


def circulant_from_column(c):
    l = c.shape[-1]
    i = np.arange(l)
    return c[(i[:, None] - i[None, :]) % l]


def average_wrapped(T, ax_i: int, ax_j: int):
    """Replace, for every other index, the l x l slice on axes (ax_i, ax_j) by the
    average over its wrapped diagonals ((i - j) mod l fixed): the Frobenius-nearest
    circulant of that slice (each wrapped diagonal is one free parameter)."""
    Tm = np.moveaxis(T, (ax_i, ax_j), (-2, -1))
    l = Tm.shape[-1]
    i = np.arange(l)
    dmat = (i[:, None] - i[None, :]) % l
    out = np.empty_like(Tm)
    for dd in range(l):
        sel = dmat == dd
        out[..., sel] = Tm[..., sel].mean(axis=-1, keepdims=True)
    return np.moveaxis(out, (-2, -1), (ax_i, ax_j))


def bttb_full(shape, k: float, d: float):
    """d^3 G between every pair of box voxels: [3][nz][ny][nx][3][nz][ny][nx], zero self term."""
    nz, ny, nx = shape
    Ks = kernel_signed(shape, k, d)  # [6][2nz-1][2ny-1][2nx-1]
    iz, iy, ix = np.arange(nz), np.arange(ny), np.arange(nx)
    dz = (iz[:, None] - iz[None, :]) + nz - 1
    dy = (iy[:, None] - iy[None, :]) + ny - 1
    dx = (ix[:, None] - ix[None, :]) + nx - 1
    T = np.empty((3, nz, ny, nx, 3, nz, ny, nx), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            Kc = Ks[FULL[a, b]]
            blk = Kc[dz[:, None, None, :, None, None], dy[None, :, None, None, :, None],
                     dx[None, None, :, None, None, :]]
            T[a, :, :, :, b] = blk
    return T


def two_level_dense(shape, k: float, d: float, alpha_tilde_inv: complex):
    """Brute-force P = alpha~^{-1} I - C2(d^3 G) over the whole box: (3N x 3N), box order."""
    nz, ny, nx = shape
    T = bttb_full(shape, k, d)
    C1 = average_wrapped(T, 3, 7)  # x level
    C2 = average_wrapped(C1, 2, 6)  # y level
    n3 = 3 * nz * ny * nx
    P = -C2.reshape(n3, n3)
    P[np.arange(n3), np.arange(n3)] += alpha_tilde_inv
    return P


def one_level_dense(shape, k: float, d: float, alpha_tilde_inv: complex):
    """Brute-force 1-level P = alpha~^{-1} I - C1(d^3 G): only the x-level Toeplitz blocks are
    replaced by their Frobenius-nearest circulants (Sec. 3, C_B); (3N x 3N), box order."""
    nz, ny, nx = shape
    C1 = average_wrapped(bttb_full(shape, k, d), 3, 7)
    n3 = 3 * nz * ny * nx
    P = -C1.reshape(n3, n3)
    P[np.arange(n3), np.arange(n3)] += alpha_tilde_inv
    return P


def one_level_blocks(shape, k: float, d: float, alpha_tilde_inv: complex):
    """Per-mode blocks of the 1-level preconditioner: eq. Chan along x of the signed kernel, a
    DFT over x, and for each of the nx modes the dense (3 nz ny) x (3 nz ny) block
    D(wx)[(a, iz, iy), (b, jz, jy)] = alpha~^{-1} delta - lambda_ab(wx; iz - jz, iy - jy)
    (block-Toeplitz-Toeplitz-block in z and y): [nx][3 nz ny][3 nz ny]."""
    nz, ny, nx = shape
    c1 = chan_column(kernel_signed(shape, k, d))  # [6][2nz-1][2ny-1][nx]
    lam = np.fft.fft(c1, axis=3)
    iz, iy = np.arange(nz), np.arange(ny)
    dz = (iz[:, None] - iz[None, :]) + nz - 1
    dy = (iy[:, None] - iy[None, :]) + ny - 1
    m = nz * ny
    D = np.empty((nx, 3 * m, 3 * m), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            L = lam[FULL[a, b]][dz[:, None, :, None], dy[None, :, None, :]]  # [nz][ny][nz][ny][nx]
            D[:, a * m:(a + 1) * m, b * m:(b + 1) * m] = -np.moveaxis(L, 4, 0).reshape(nx, m, m)
    idx = np.arange(3 * m)
    D[:, idx, idx] += alpha_tilde_inv
    return D


def apply_one_level(vbox, mask, Dinv):
    """z = M P^{-1} (M v) for the 1-level preconditioner given by its per-mode inverse blocks."""
    m = mask.astype(np.float64)[None]
    nx = vbox.shape[3]
    V = np.fft.fft(vbox * m, axis=3)  # [3][nz][ny][nx]
    Vm = np.moveaxis(V, 3, 0).reshape(nx, -1)  # unknown order (a, iz, iy) per mode
    Z = np.einsum("xij,xj->xi", Dinv, Vm)
    Z = np.moveaxis(Z.reshape((nx,) + V.shape[:3]), 0, 3)
    return m * np.fft.ifft(Z, axis=3)


def two_level_generator(shape, k: float, d: float):
    """c2_c(qbar, pbar, s): eq. Chan along x then y of the signed kernel.

    Returns complex128 [6][2nz-1][ny][nx] (s index s + nz - 1)."""
    Ks = kernel_signed(shape, k, d)  # [6][2nz-1][2ny-1][2nx-1]
    c1 = chan_column(Ks)  # along x -> [6][2nz-1][2ny-1][nx]
    c2 = chan_column(np.moveaxis(c1, 2, -1))  # along y -> [6][2nz-1][nx][ny]
    return np.moveaxis(c2, -1, 2)


def two_level_blocks(shape, k: float, d: float, alpha_tilde_inv: complex):
    """Per-mode blocks B(wy, wx) = alpha~^{-1} I - [lambda_ab(w, iz - jz)]: [ny][nx][3nz][3nz].

    Unknown order inside a block is (component a, z index iz), a-major.
    """
    nz, ny, nx = shape
    c2 = two_level_generator(shape, k, d)
    lam = np.fft.fft2(c2, axes=(2, 3))  # [6][2nz-1][ny][nx]
    iz = np.arange(nz)
    ds = (iz[:, None] - iz[None, :]) + nz - 1
    B = np.empty((ny, nx, 3 * nz, 3 * nz), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            L = lam[FULL[a, b]][ds]  # [nz][nz][ny][nx]
            B[:, :, a * nz:(a + 1) * nz, b * nz:(b + 1) * nz] = -np.moveaxis(L, (0, 1), (2, 3))
    idx = np.arange(3 * nz)
    B[:, :, idx, idx] += alpha_tilde_inv
    return B


def invert_blocks(B):
    """Explicit inverses of every mode block (LU with partial pivoting per block)."""
    out = np.empty_like(B)
    eye = np.eye(B.shape[-1], dtype=B.dtype)
    for j in range(B.shape[0]):
        for i in range(B.shape[1]):
            lu = sla.lu_factor(B[j, i])
            out[j, i] = sla.lu_solve(lu, eye)
    return out


def apply_blocks(vbox, mask, Binv):
    """z = M P^{-1} (M v) with P given by its per-mode inverse blocks."""
    m = mask.astype(np.float64)[None]
    nz = vbox.shape[1]
    V = np.fft.fft2(vbox * m, axes=(2, 3))  # [3][nz][ny][nx]
    Vm = np.moveaxis(V, (2, 3), (0, 1)).reshape(V.shape[2], V.shape[3], 3 * nz)
    Z = np.einsum("yxij,yxj->yxi", Binv, Vm)
    Z = np.moveaxis(Z.reshape(V.shape[2], V.shape[3], 3, nz), (0, 1), (2, 3))
    return m * np.fft.ifft2(Z, axes=(2, 3))


def apply_dense(vbox, mask, P):
    """z = M P^{-1} (M v) with the dense brute-force P (LU solve)."""
    m = mask.astype(np.float64)[None]
    z = np.linalg.solve(P, (vbox * m).ravel()).reshape(vbox.shape)
    return m * z


def occupied_layers(mask):
    """(z0, z1): the first and one-past-last z layer holding an occupied voxel.

    The paper's grid is the smallest box around the body (Sec. 4), so its dense (z) level
    spans exactly these layers; a box with extra air layers keeps that preconditioner."""
    zs = np.flatnonzero(np.asarray(mask).reshape(mask.shape[0], -1).any(axis=1))
    return int(zs[0]), int(zs[-1]) + 1


def blocks_for_mask(mask, k: float, d: float, alpha_tilde_inv: complex):
    """(z0, inverse blocks) of the 2-level preconditioner on the occupied layers of ``mask``."""
    z0, z1 = occupied_layers(mask)
    shape = (z1 - z0,) + tuple(mask.shape[1:])
    return z0, invert_blocks(two_level_blocks(shape, k, d, alpha_tilde_inv))


def apply_blocks_layers(vbox, mask, Binv, z0: int):
    """z = M P^{-1} (M v) with P built on layers z0 .. z0 + bz - 1 (bz = Binv's z extent); the
    layers outside hold only air, so they come out zero."""
    bz = Binv.shape[-1] // 3
    out = np.zeros_like(vbox, dtype=np.complex128)
    out[:, z0:z0 + bz] = apply_blocks(vbox[:, z0:z0 + bz], mask[z0:z0 + bz], Binv)
    return out


def diag_correction(eps, mask, kd: float, S: float, alpha_tilde_inv: complex):
    """Delta = D - alpha~^{-1} I on the box (0 in air): the part of the true diagonal
    D = diag(1/alpha_j) that the circulant preconditioner's constant diagonal misses (Sec. 1,
    P = D~ + C; Sec. 5, circulant-plus-diagonal)."""
    from . import physics
    occ = np.asarray(mask).astype(bool)
    return np.where(occ, physics.alpha_inv_masked(eps, mask, kd, S) - alpha_tilde_inv, 0.0)


def apply_plus_diagonal(vbox, apply_B, delta, steps: int):
    """z ~ (D + C)^{-1} v for the circulant-plus-diagonal P = D + C = B + Delta, where
    B = alpha~^{-1} I + C is the circulant preconditioner, applied as Q = M B^{-1} M
    (apply_B), and Delta = D - alpha~^{-1} I: the fixed point of z = Q (v - Delta z), i.e.
    (Q^{-1} + Delta)^{-1} v on the occupied voxels, taken from z_0 = Q v in `steps` more steps
    (the Neumann series of (I + Q Delta)^{-1} Q truncated after steps + 1 terms).  steps = 0
    is the circulant preconditioner itself."""
    z = apply_B(vbox)
    for _ in range(steps):
        z = apply_B(vbox - delta[None] * z)
    return z
