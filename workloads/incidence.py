"""Incident plane waves: propagation directions and real unit polarisations.

Each wave is given by a unit direction ``dir`` and a real unit polarisation
``pol`` orthogonal to it (the paper's d and E_0 in the LDR polarisability,
Sec. 2.1).  Only geometry of unit vectors is done here.
"""

from __future__ import annotations

import numpy as np


def plane_wave_z(pols=("x",)):
    """Waves travelling along +z with the listed polarisations ('x' and/or 'y')."""
    unit = {"x": (1.0, 0.0, 0.0), "y": (0.0, 1.0, 0.0)}
    dirs = np.array([(0.0, 0.0, 1.0)] * len(pols))
    pol = np.array([unit[p] for p in pols])
    return dirs, pol


def _orthonormal_pair(dvec):
    ez = np.array([0.0, 0.0, 1.0])
    e1 = np.cross(ez, dvec)
    nrm = np.linalg.norm(e1)
    if nrm < 1e-8:
        e1 = np.array([1.0, 0.0, 0.0])
    else:
        e1 = e1 / nrm
    e2 = np.cross(dvec, e1)
    e2 /= np.linalg.norm(e2)
    return e1, e2


def batch_directions(dirs_raw):
    """Turn raw 3-vectors into (dir, pol) pairs: two polarisations per direction.

    For each direction d, e1 = normalise(z x d) (x if d is along z) and
    e2 = d x e1; the returned arrays interleave (d, e1), (d, e2).
    """
    dirs, pols = [], []
    for v in np.asarray(dirs_raw, dtype=np.float64):
        dv = v / np.linalg.norm(v)
        e1, e2 = _orthonormal_pair(dv)
        dirs += [dv, dv]
        pols += [e1, e2]
    return np.array(dirs), np.array(pols)


def random_directions(n_dirs: int, rng):
    """``n_dirs`` directions uniform on the sphere (normalised Gaussians), 2 pols each."""
    raw = rng.normal(size=(n_dirs, 3))
    return batch_directions(raw)
