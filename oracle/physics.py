"""Polarisability and Green tensor (paper Sec. 2 and 2.1).  Test infrastructure only."""

from __future__ import annotations

import numpy as np

# Lattice-dispersion-relation coefficients (Sec. 2.1, definitions under eq. CM).
B1 = -1.891531
B2 = 0.1648469
B3 = -1.7700004

# Order of the six unique tensor components (Algorithm 1): xx, xy, xz, yy, yz, zz.
COMP6 = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def lattice_S(direction, polarisation) -> float:
    """S = sum_j (d_j E_j)^2 for unit incident direction d and polarisation E (Sec. 2.1)."""
    d = np.asarray(direction, dtype=np.float64)
    e = np.asarray(polarisation, dtype=np.float64)
    return float(np.sum((d * e) ** 2))


def alpha_inv(eps, kd: float, S: float):
    """Inverse LDR polarisability with the voxel volume omitted (Sec. 2.1).

    alpha^CM = (3 / 4 pi) (eps - 1) / (eps + 2) and
    alpha^LDR = alpha^CM / (1 + alpha^CM [(b1 + m^2 b2 + m^2 b3 S)(k d)^2 - (2i/3)(k d)^3]),
    so 1 / alpha^LDR = 1 / alpha^CM + (b1 + eps b2 + eps b3 S)(k d)^2 - (2i/3)(k d)^3
    with m^2 = eps.  Works elementwise on arrays.
    """
    eps = np.asarray(eps, dtype=np.complex128)
    inv_cm = (4.0 * np.pi / 3.0) * (eps + 2.0) / (eps - 1.0)
    return inv_cm + (B1 + eps * B2 + eps * B3 * S) * kd ** 2 - (2j / 3.0) * kd ** 3


def alpha_inv_masked(eps, mask, kd: float, S: float):
    """:func:`alpha_inv` on occupied voxels, 0 in air (where it is undefined for eps = 1)."""
    occ = np.asarray(mask).astype(bool)
    safe = np.where(occ, np.asarray(eps, dtype=np.complex128), 2.0)
    return np.where(occ, alpha_inv(safe, kd, S), 0.0)


def alpha_tilde_inv(eps, mask, kd: float, S: float, variant: str = "mean_eps"):
    """The constant diagonal alpha~^{-1} of the circulant preconditioner P = D~ + C (Sec. 1,
    Sec. 3.1), from the occupied voxels' permittivities, in one of three readings:

    * "mean_eps":   alpha^{-1} of the mean occupied permittivity;
    * "mean_alpha": the mean of alpha^{-1} over the occupied voxels (the diagonal averaged);
    * "mode":       alpha^{-1} of the most frequent occupied permittivity (the paper's modal
                    average of the diagonal, over the body); a tie goes to the smallest value
                    (real part, then imaginary part), which no voxel ordering affects.

    All three equal the body's own value for a homogeneous body.
    """
    occ = np.asarray(mask).astype(bool).ravel()
    e = np.asarray(eps, dtype=np.complex128).ravel()[occ]
    if variant == "mean_eps":
        return complex(alpha_inv(e.mean(), kd, S))
    if variant == "mean_alpha":
        return complex(alpha_inv(e, kd, S).mean())
    if variant == "mode":
        vals, counts = np.unique(e, return_counts=True)
        top = counts.max()
        cand = sorted((v.real, v.imag) for v, c in zip(vals, counts) if c == top)
        return complex(alpha_inv(complex(*cand[0]), kd, S))
    raise ValueError(f"unknown variant {variant!r}")


def dalpha_inv_deps(eps, kd: float, S: float):
    """d(1/alpha^LDR)/d eps of :func:`alpha_inv` (holomorphic in eps)."""
    eps = np.asarray(eps, dtype=np.complex128)
    return -4.0 * np.pi / (eps - 1.0) ** 2 + (B2 + B3 * S) * kd ** 2


def green(R, k: float):
    """Dyadic Green tensor of Sec. 2 at displacement(s) R (shape (..., 3)) -> (..., 3, 3).

    G = e^{ikr}/r [k^2 (I - rr^T) + (ikr - 1)/r^2 (I - 3 rr^T)], r = |R|, with
    G := 0 at R = 0 (the self term is carried by the polarisability,
    Algorithm 1 skips r = 0).
    """
    R = np.asarray(R, dtype=np.float64)
    r = np.sqrt(np.sum(R * R, axis=-1))
    zero = r == 0.0
    rs = np.where(zero, 1.0, r)
    rh = R / rs[..., None]
    outer = rh[..., :, None] * rh[..., None, :]
    eye = np.eye(3)
    ph = np.exp(1j * k * rs) / rs
    term1 = (k * k) * (eye - outer)
    term2 = ((1j * k * rs - 1.0) / rs ** 2)[..., None, None] * (eye - 3.0 * outer)
    G = ph[..., None, None] * (term1 + term2)
    G[zero] = 0.0
    return G


def green6(R, k: float):
    """The six unique components of :func:`green` stacked last: (..., 6)."""
    G = green(R, k)
    return np.stack([G[..., a, b] for a, b in COMP6], axis=-1)
