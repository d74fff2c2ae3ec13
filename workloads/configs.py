"""The five benchmark workloads (synthetic hexagonal ice prisms) and their seeds.

All prisms use the grid mode of :func:`hex_prism_grid` (cubic grid, longest
extent spans it).  Refractive index 1.31 is ice in the visible; eps = m^2.

* c1: x = 2, aspect 1, 16^3, m = 1.31, +z / x-pol, tol 1e-6.
* c2: x = 20, aspect 1, 128^3, m = 1.31, +z / (x-pol, y-pol), tol 1e-5.
* c3: x = 40, aspect 2, 256^3, m = 1.31+0.001i (and 1.78), +z / x-pol, tol 1e-5.
* c4: 16 prisms from ``default_rng(1903)``: per prism aspect ~ U[0.5, 2] then
  x ~ U[5, 20] (drawn in that order); grid = element of {32,...,96} nearest to
  32 + 64 (x - 5) / 15; then 64 Gaussian directions, 2 polarisations each.
* c5: x = 10, aspect 1, 64^3, eps_j = 1.7161 (1 + delta_j), delta_j ~ U[-0.05, 0.05]
  from ``default_rng(9802)`` over occupied voxels in C order; dense check grid
  12^3 at the same k d (x = 1.875).
* plates: the paper's Sec. 4 experiment, hexagonal plates L/a = 0.1, 0.2 with
  mu = 1.2 ... 2 and x = 10 ... 100 at lambda / (mu d) = 10, lit by (0, 0, 1) e^{ikx};
  each box is the fitted grid grown at its high ends to the next 2-3-5-7-smooth size
  (air voxels only), since the FFT lengths are 2 n per axis.
"""

from __future__ import annotations

import numpy as np

import math

from .geometry import SQRT3, Scatterer, hex_prism_fit, hex_prism_grid
from .incidence import plane_wave_z, random_directions

C4_GRIDS = (32, 40, 48, 56, 64, 72, 80, 96)


def config_c1():
    s = hex_prism_grid(2.0, 1.0, 16, 1.31, name="c1_hex16")
    dirs, pols = plane_wave_z(("x",))
    return dict(name="c1", scatterer=s, dirs=dirs, pols=pols, tol=1e-6, restart=30)


def config_c2():
    s = hex_prism_grid(20.0, 1.0, 128, 1.31, name="c2_hex128")
    dirs, pols = plane_wave_z(("x", "y"))
    return dict(name="c2", scatterer=s, dirs=dirs, pols=pols, tol=1e-5, restart=30)


def config_c3(case: int = 0):
    m = 1.31 + 0.001j if case == 0 else 1.78
    s = hex_prism_grid(40.0, 2.0, 256, m, name=f"c3_hex256_m{case}")
    dirs, pols = plane_wave_z(("x",))
    return dict(name="c3", scatterer=s, dirs=dirs, pols=pols, tol=1e-5, restart=30)


def c4_grid_for(x: float) -> int:
    target = 32.0 + 64.0 * (x - 5.0) / 15.0
    return min(C4_GRIDS, key=lambda g: (abs(g - target), g))


def config_c4(n_prisms: int = 16, n_dirs: int = 64, seed: int = 1903):
    rng = np.random.default_rng(seed)
    prisms = []
    for i in range(n_prisms):
        aspect = rng.uniform(0.5, 2.0)
        x = rng.uniform(5.0, 20.0)
        g = c4_grid_for(x)
        s = hex_prism_grid(x, aspect, g, 1.31, name=f"c4_p{i}_g{g}")
        dirs, pols = random_directions(n_dirs, rng)
        prisms.append(dict(scatterer=s, dirs=dirs, pols=pols))
    return dict(name="c4", prisms=prisms, tol=1e-5, restart=30)


def _jitter_eps(s, seed):
    rng = np.random.default_rng(seed)
    occ = s.mask.astype(bool)
    delta = rng.uniform(-0.05, 0.05, size=int(occ.sum()))
    eps = np.ones(s.mask.shape, dtype=np.complex128)
    eps[occ] = 1.7161 * (1.0 + delta)
    s.eps = eps
    return s


def config_c5():
    s = _jitter_eps(hex_prism_grid(10.0, 1.0, 64, 1.31, name="c5_hex64"), 9802)
    dirs, pols = plane_wave_z(("x",))
    fd_rng = np.random.default_rng(4242)
    occ_idx = np.flatnonzero(s.mask.ravel())
    fd_voxels = np.sort(fd_rng.choice(occ_idx, size=32, replace=False))
    return dict(name="c5", scatterer=s, dirs=dirs, pols=pols, tol=1e-5, restart=30,
                fd_voxels=fd_voxels)


def config_c5_dense():
    s = _jitter_eps(hex_prism_grid(1.875, 1.0, 12, 1.31, name="c5_hex12"), 9802)
    dirs, pols = plane_wave_z(("x",))
    return dict(name="c5_dense", scatterer=s, dirs=dirs, pols=pols, tol=1e-10, restart=30)


PLATE_MU = (1.2, 1.4, 1.6, 1.8, 2.0)
PLATE_X = (10, 20, 30, 40, 60, 80, 100)


def smooth7(n: int) -> int:
    """Smallest m >= n whose only prime factors are 2, 3, 5 and 7."""
    m = max(1, int(n))
    while True:
        k = m
        for f in (2, 3, 5, 7):
            while k % f == 0:
                k //= f
        if k == 1:
            return m
        m += 1


def plate_fit_rounding(l_over_a: float, mu: float, x: float, total: float) -> str:
    """The box rounding ("ceil" or "round") whose voxel total is closer to ``total`` (the
    paper prints its totals to two digits and neither rule reproduces all of them)."""
    d = 2.0 * math.pi / float(x) / (10.0 * float(mu))
    best = None
    for rnd in ("ceil", "round"):
        f = math.ceil if rnd == "ceil" else (lambda v: max(1, int(round(v))))
        n = 1
        for e in (2.0, SQRT3, float(l_over_a)):
            n *= max(1, f(e / d - 1e-12))
        err = abs(n / float(total) - 1.0)
        if best is None or err < best[0]:
            best = (err, rnd)
    return best[1]


def plate_case(l_over_a: float, mu: float, x: float, rounding: str = "ceil"):
    """One plate of the Sec. 4 sweep: the fitted voxelisation, zero-padded (air) at the high
    end of each axis to 7-smooth dimensions, and the incident wave (0, 0, 1) e^{ikx}."""
    f = hex_prism_fit(float(x), float(l_over_a), float(mu), rounding=rounding)
    nz, ny, nx = f.mask.shape
    pz, py, px = smooth7(nz), smooth7(ny), smooth7(nx)
    mask = np.zeros((pz, py, px), dtype=np.uint8)
    eps = np.ones((pz, py, px), dtype=np.complex128)
    mask[:nz, :ny, :nx] = f.mask
    eps[:nz, :ny, :nx] = f.eps
    meta = dict(f.meta, fit_shape=(nz, ny, nx), fit_total=nz * ny * nx)
    s = Scatterer(f"plate_la{l_over_a}_mu{mu}_x{x}", mask, eps, k=f.k, d=f.d, meta=meta)
    dirs = np.array([[1.0, 0.0, 0.0]])
    pols = np.array([[0.0, 0.0, 1.0]])
    return dict(name="plate", scatterer=s, dirs=dirs, pols=pols, tol=1e-5, restart=30)
