"""Shared helpers for GPU tests: build torch inputs from workloads, compare with the oracle."""

import numpy as np

import workloads as w


def torch_inputs(s):
    import torch
    return torch.from_numpy(s.mask).cuda(), torch.from_numpy(s.eps).cuda()


def make_problem(s, **kw):
    from paper_1903_09802_amd.dda import Problem
    m, e = torch_inputs(s)
    return Problem(m, e, s.k, s.d, **kw)


def rand_field(shape, nrhs, seed, mask=None):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(nrhs, 3) + shape) + 1j * rng.normal(size=(nrhs, 3) + shape)
    if mask is not None:
        x = x * mask[None, None]
    return x


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def random_waves(n, seed):
    rng = np.random.default_rng(seed)
    return w.random_directions((n + 1) // 2, rng)


def oracle_precond(s, s_bar=0.0, variant="mean_eps"):
    """v -> M P^{-1} M v of the oracle's 2-level preconditioner on the occupied z layers, with
    alpha~^{-1} averaged over the occupied voxels as ``variant`` says (by default of the mean
    occupied permittivity: what build_preconditioner(s_bar) builds with alpha_avg 0)."""
    from oracle import circulant, physics
    ati = physics.alpha_tilde_inv(s.eps, s.mask, s.k * s.d, s_bar, variant)
    z0, Binv = circulant.blocks_for_mask(s.mask, s.k, s.d, ati)
    return lambda v: circulant.apply_blocks_layers(v, s.mask, Binv, z0)
