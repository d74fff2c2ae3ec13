"""Voxelised scatterers on a uniform grid (the paper's Sec. 2.2 discretisation).

Conventions used throughout the project:

* arrays are C-ordered ``[nz][ny][nx]`` (x fastest), matching the x / y / z
  levels of the block-Toeplitz structure (x = level 1, y = level 2, z = level 3);
* lengths are in units of the circumradius ``a`` of the hexagonal face, so the
  wavenumber is ``k = x / a = x`` for size parameter ``x = k a`` (Sec. 4);
* voxel ``(ix, iy, iz)`` has its centre at ``((ix - (nx-1)/2) d, (iy - (ny-1)/2) d,
  (iz - (nz-1)/2) d)``, i.e. the grid is centred on the origin;
* ``eps`` holds the relative permittivity at occupied voxels and 1 (vacuum) in
  air.  Air voxels carry no unknowns (the polarisation vanishes where the
  susceptibility does, Sec. 2 below the polarisation integral equation).

The hexagonal prism has its axis along z and a vertex of the hexagon on +x
(vertices at 0, 60, ..., 300 degrees), as in Fig. 3 of the paper.  A voxel is
occupied when its centre lies inside the closed prism (tolerance 1e-9 d).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQRT3 = math.sqrt(3.0)


@dataclass
class Scatterer:
    """A voxelised body plus the wavenumber it is illuminated at."""

    name: str
    mask: np.ndarray  # uint8 [nz][ny][nx], 1 = occupied
    eps: np.ndarray  # complex128 [nz][ny][nx], 1 in air
    k: float  # wavenumber (1/length)
    d: float  # voxel edge length
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.mask.shape  # (nz, ny, nx)

    @property
    def nx(self):
        return self.mask.shape[2]

    @property
    def ny(self):
        return self.mask.shape[1]

    @property
    def nz(self):
        return self.mask.shape[0]

    @property
    def n_occ(self):
        return int(self.mask.sum())


def voxel_centres(nx: int, ny: int, nz: int, d: float):
    """Centre coordinates of every voxel as three broadcastable arrays (z, y, x order)."""
    x = (np.arange(nx) - (nx - 1) / 2.0) * d
    y = (np.arange(ny) - (ny - 1) / 2.0) * d
    z = (np.arange(nz) - (nz - 1) / 2.0) * d
    return z[:, None, None], y[None, :, None], x[None, None, :]


def _hex_inside(X, Y, Z, a, L, tol):
    ax, ay, az = np.abs(X), np.abs(Y), np.abs(Z)
    return (
        (ay <= SQRT3 / 2.0 * a + tol)
        & (SQRT3 * ax + ay <= SQRT3 * a + tol)
        & (az <= L / 2.0 + tol)
    )


def _fill_eps(mask: np.ndarray, eps_val) -> np.ndarray:
    eps = np.ones(mask.shape, dtype=np.complex128)
    eps[mask.astype(bool)] = eps_val
    return eps


def hex_prism_grid(size_param: float, aspect: float, g: int, m_index: complex,
                   name: str = "hex") -> Scatterer:
    """Hexagonal prism on a cubic g x g x g grid.

    ``aspect`` is length / diameter, so the prism length is ``L = aspect * 2a``.
    The voxel edge is ``d = max(2a, L) / g`` so the longest extent spans the
    grid; ``m_index`` is the complex refractive index (eps = m^2).
    """
    a = 1.0
    L = aspect * 2.0 * a
    d = max(2.0 * a, L) / g
    Z, Y, X = voxel_centres(g, g, g, d)
    inside = _hex_inside(X, Y, Z, a, L, 1e-9 * d)
    mask = np.ascontiguousarray(inside.astype(np.uint8))
    eps_val = complex(m_index) ** 2
    return Scatterer(name, mask, _fill_eps(mask, eps_val), k=size_param / a, d=d,
                     meta=dict(kind="hex_prism_grid", x=size_param, aspect=aspect,
                               g=g, m=complex(m_index)))


def hex_prism_fit(size_param: float, l_over_a: float, mu: float,
                  rounding: str = "ceil", name: str = "plate") -> Scatterer:
    """Hexagonal plate discretised as in the paper's Sec. 4 experiments.

    The voxel edge follows the resolution rule lambda / (mu d) = 10 (Sec. 2.2)
    and the grid is the smallest box around the 2a x sqrt(3)a x L plate, with
    each dimension rounded up (``"ceil"``) or to nearest (``"round"``).
    """
    a = 1.0
    k = size_param / a
    lam = 2.0 * math.pi / k
    d = lam / (10.0 * mu)
    L = l_over_a * a
    ext = (2.0 * a, SQRT3 * a, L)
    rnd = math.ceil if rounding == "ceil" else (lambda v: max(1, int(round(v))))
    nx, ny, nz = (max(1, rnd(e / d - 1e-12)) for e in ext)
    Z, Y, X = voxel_centres(nx, ny, nz, d)
    inside = _hex_inside(X, Y, Z, a, L, 1e-9 * d)
    mask = np.ascontiguousarray(inside.astype(np.uint8))
    return Scatterer(name, mask, _fill_eps(mask, mu * mu), k=k, d=d,
                     meta=dict(kind="hex_prism_fit", x=size_param, l_over_a=l_over_a,
                               mu=mu, rounding=rounding))


def sphere_grid(k_radius: float, g: int, m_index: complex, name: str = "sphere") -> Scatterer:
    """Sphere of radius 1 voxelised on a g^3 grid with d = 2 / g; ``k = k_radius``."""
    r = 1.0
    d = 2.0 * r / g
    Z, Y, X = voxel_centres(g, g, g, d)
    inside = X * X + Y * Y + Z * Z <= r * r + 1e-9 * d
    mask = np.ascontiguousarray(inside.astype(np.uint8))
    return Scatterer(name, mask, _fill_eps(mask, complex(m_index) ** 2), k=k_radius, d=d,
                     meta=dict(kind="sphere", g=g, m=complex(m_index)))


def cuboid_grid(nx: int, ny: int, nz: int, k: float, d: float, m_index: complex,
                name: str = "cuboid") -> Scatterer:
    """Fully occupied box (a homogeneous cuboid: the case where the system is exactly BTTB)."""
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    return Scatterer(name, mask, _fill_eps(mask, complex(m_index) ** 2), k=k, d=d,
                     meta=dict(kind="cuboid"))


def random_mask(nx: int, ny: int, nz: int, fill: float, seed: int, k: float, d: float,
                eps_mean: complex = 1.7161, eps_jitter: float = 0.0,
                name: str = "random") -> Scatterer:
    """Random occupancy with optional per-voxel permittivity jitter (test inputs)."""
    rng = np.random.default_rng(seed)
    mask = (rng.random((nz, ny, nx)) < fill).astype(np.uint8)
    if mask.sum() == 0:
        mask.flat[0] = 1
    eps = np.ones(mask.shape, dtype=np.complex128)
    occ = mask.astype(bool)
    jit = eps_jitter * (rng.random(occ.sum()) * 2 - 1) + 1j * eps_jitter * 0.1 * rng.random(occ.sum())
    eps[occ] = eps_mean * (1.0 + jit)
    return Scatterer(name, np.ascontiguousarray(mask), eps, k=k, d=d,
                     meta=dict(kind="random", fill=fill, seed=seed))
