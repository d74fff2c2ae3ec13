"""FFT form of the BTTB product (paper Sec. 1 and 2.2).  Test infrastructure only.

The off-diagonal part of the DDA matrix is a 3-level block-Toeplitz convolution:
(T x)_i = sum_j K(i - j) x_j with K(p, q, s) = d^3 G(p d, q d, s d) for signed
voxel offsets |p| < nx, |q| < ny, |s| < nz and K(0) = 0 (Algorithm 1 defines G by
one "row"; here the kernel is evaluated directly at every signed offset).  A
circular convolution of length 2 nx (etc.) with the input zero-padded to that
length reproduces the linear one on the first nx outputs, so one FFT of the
embedded kernel and a forward / inverse FFT per component give the product in
O(N log N) (the paper's premise, Sec. 1).  The offset of exactly +-nx never
occurs and is left at zero in the embedding.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .physics import COMP6, alpha_inv_masked, green6


def kernel_signed(shape, k: float, d: float, part: str = "full"):
    """K_c(p, q, s) for c in the six components, p in (-nx, nx) etc.

    Returns complex128 [6][2nz-1][2ny-1][2nx-1]; index (s + nz - 1, q + ny - 1, p + nx - 1).
    ``part='imag'`` gives d^3 Im G instead (the kernel of the scattering sum).
    """
    nz, ny, nx = shape
    p = np.arange(-(nx - 1), nx) * d
    q = np.arange(-(ny - 1), ny) * d
    s = np.arange(-(nz - 1), nz) * d
    S, Q, P = np.meshgrid(s, q, p, indexing="ij")
    R = np.stack([P, Q, S], axis=-1)
    K = (d ** 3) * green6(R, k)
    if part == "imag":
        K = K.imag.astype(np.complex128)
    return np.moveaxis(K, -1, 0).copy()


def kernel_padded_fft(shape, k: float, d: float, part: str = "full", workers: int = -1):
    """FFT of the circulant embedding of :func:`kernel_signed`: complex128 [6][2nz][2ny][2nx]."""
    nz, ny, nx = shape
    Ks = kernel_signed(shape, k, d, part)
    emb = np.zeros((6, 2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
    iz = np.arange(-(nz - 1), nz) % (2 * nz)
    iy = np.arange(-(ny - 1), ny) % (2 * ny)
    ix = np.arange(-(nx - 1), nx) % (2 * nx)
    emb[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]] = Ks
    return sfft.fftn(emb, axes=(1, 2, 3), workers=workers)


def convolve(xbox, Khat, workers: int = -1):
    """(T x) restricted to the box: sum_j K(i - j) x_j for all voxels i (no mask, no diagonal)."""
    _, nz, ny, nx = xbox.shape
    Lz, Ly, Lx = 2 * nz, 2 * ny, 2 * nx
    X = sfft.fftn(xbox, s=(Lz, Ly, Lx), axes=(1, 2, 3), workers=workers)
    full = np.zeros((3, 3), dtype=int)
    for c, (a, b) in enumerate(COMP6):
        full[a, b] = full[b, a] = c
    Y = np.empty_like(X)
    for a in range(3):
        Y[a] = Khat[full[a, 0]] * X[0] + Khat[full[a, 1]] * X[1] + Khat[full[a, 2]] * X[2]
    y = sfft.ifftn(Y, axes=(1, 2, 3), workers=workers)
    return y[:, :nz, :ny, :nx]


def fft_matvec(xbox, mask, eps, k: float, d: float, S: float, Khat=None, workers: int = -1):
    """Full-box DDA operator: y = M (alpha^{-1} x - T(M x)) + (1 - M) x.

    On occupied voxels this is the dense matrix of :mod:`oracle.system` applied
    to the occupied entries; air entries are passed through unchanged, so a
    vector that is zero in air stays zero in air.
    """
    if Khat is None:
        Khat = kernel_padded_fft(mask.shape, k, d, workers=workers)
    m = mask.astype(np.float64)[None]
    conv = convolve(xbox * m, Khat, workers=workers)
    ainv = alpha_inv_masked(eps, mask, k * d, S)[None]
    return m * (ainv * xbox - conv) + (1.0 - m) * xbox
