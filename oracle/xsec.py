r"""Cross sections of the solved dipole array.  Test infrastructure only.

The paper reports no cross sections; these are the Draine-Flatau expressions
(the DDA formulation the paper follows, Sec. 2.1) rewritten for its scaling, in
which the unknown c is a polarisation density and the voxel volume d^3 is
omitted from the polarisability (so the dipole moment is d^3 c).  With
|E_0| = 1:

    C_ext = 4 pi k d^3 sum_i Im(E_inc,i^* . c_i)
    C_abs = 4 pi k d^3 sum_i |c_i|^2 (-Im alpha_i^{-1} - (2/3)(k d)^3)
    C_sca = k^4 d^6 \int |sum_i (I - n n^T) c_i e^{-i k n . r_i}|^2 dOmega
          = 4 pi k d^3 [(2/3)(k d)^3 sum_i |c_i|^2 + sum_{i != j} c_i^H (d^3 Im G_ij) c_j]

The last identity uses \int (I - n n^T) e^{i k n . R} dOmega = (4 pi / k^3) Im G(R),
Im G(0) = (2/3) k^3 I.  Both the far-field quadrature and the Im G double sum
are implemented so each pins the other; C_ext = C_abs + C_sca for the exact
solution (optical theorem).
"""

from __future__ import annotations

import numpy as np

from .fftmatvec import convolve, kernel_padded_fft
from .physics import alpha_inv_masked, green, lattice_S
from .system import centres, incident_field


def c_ext(cbox, mask, k, d, direction, polarisation):
    E = incident_field(mask, k, d, direction, polarisation)
    return float(4.0 * np.pi * k * d ** 3 * np.sum(np.imag(np.conj(E) * cbox)))


def c_abs(cbox, mask, eps, k, d, direction, polarisation):
    ainv = alpha_inv_masked(eps, mask, k * d, lattice_S(direction, polarisation))
    w = (-np.imag(ainv) - (2.0 / 3.0) * (k * d) ** 3) * mask
    return float(4.0 * np.pi * k * d ** 3 * np.sum(np.sum(np.abs(cbox) ** 2, axis=0) * w))


def c_sca_imag_sum(cbox, mask, k, d, workers=-1):
    """Scattering cross section from the Im G double sum, evaluated by FFT convolution."""
    KhI = kernel_padded_fft(mask.shape, k, d, part="imag", workers=workers)
    cm = cbox * mask[None]
    u = convolve(cm, KhI, workers=workers)
    cross = np.real(np.sum(np.conj(cm) * u))
    self_term = (2.0 / 3.0) * (k * d) ** 3 * np.sum(np.abs(cm) ** 2)
    return float(4.0 * np.pi * k * d ** 3 * (self_term + cross))


def c_sca_imag_dense(cbox, mask, k, d):
    """Same double sum, pair by pair (small grids only)."""
    occ = mask.astype(bool).ravel()
    r = centres(mask.shape, d).reshape(-1, 3)[occ]
    c = np.stack([cbox[a].ravel()[occ] for a in range(3)], axis=-1)  # [n][3]
    ImG = np.imag(green(r[:, None, :] - r[None, :, :], k))  # zero self term
    cross = np.einsum("ia,ijab,jb->", np.conj(c), ImG, c).real * d ** 3
    self_term = (2.0 / 3.0) * (k * d) ** 3 * np.sum(np.abs(c) ** 2)
    return float(4.0 * np.pi * k * d ** 3 * (self_term + cross))


def c_sca_farfield(cbox, mask, k, d, n_theta=48, n_phi=96):
    """Scattering cross section by quadrature of the far field over the unit sphere
    (Gauss-Legendre in cos(theta), trapezoid in phi)."""
    occ = mask.astype(bool).ravel()
    r = centres(mask.shape, d).reshape(-1, 3)[occ]
    c = np.stack([cbox[a].ravel()[occ] for a in range(3)], axis=-1)
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    phi = np.arange(n_phi) * (2.0 * np.pi / n_phi)
    total = 0.0
    for ct, wt in zip(mu, wmu):
        st = np.sqrt(1.0 - ct * ct)
        n = np.stack([st * np.cos(phi), st * np.sin(phi), np.full_like(phi, ct)], axis=-1)
        ph = np.exp(-1j * k * (n @ r.T))  # [phi][voxel]
        F = ph @ c  # [phi][3] = sum_i c_i e^{-ik n.r_i}
        F = F - n * np.sum(n * F, axis=-1, keepdims=True)
        total += wt * np.sum(np.abs(F) ** 2) * (2.0 * np.pi / n_phi)
    return float(k ** 4 * d ** 6 * total)


def cross_sections(cbox, mask, eps, k, d, direction, polarisation, workers=-1):
    """(C_ext, C_abs, C_sca) with C_sca from the Im G double sum."""
    return (c_ext(cbox, mask, k, d, direction, polarisation),
            c_abs(cbox, mask, eps, k, d, direction, polarisation),
            c_sca_imag_sum(cbox, mask, k, d, workers=workers))
