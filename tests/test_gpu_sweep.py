"""Inversion of the 2-level preconditioner's symmetric blocks by the blocked symmetric sweep
(its four kernels: the matrix held on chip, tiles streamed through memory with 32- or
16-pivot panels, and the vector kernel) against pivoted Gauss-Jordan (the same products to
rounding), its fallback to Gauss-Jordan (bit for bit), and both against the oracle."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, rel_err, to_dev

pytestmark = pytest.mark.gpu

# tile rows / panels: n2 = 3 nz / 2 of 3, 18, 36, 108, 144, 192 (one to twelve 16-pivot panels,
# a partial last panel; odd tile counts pad the 32-pivot kernel with an identity tile), and
# 384.  "auto" takes the on-chip kernel up to 45 stored tiles in FP64 (order 144) and 90 in
# FP32 (order 192), the 32-pivot streaming kernel above where its panel fits the LDS (FP64 up
# to order 256); at 384 FP64 takes the 16-pivot streaming kernel, and the vector kernel
# 8-pivot panels.
SHAPES = [(2, 6, 5), (12, 4, 6), (24, 4, 3), (72, 3, 4), (96, 2, 3), (128, 2, 3)]


def _apply(s, nrhs, fp32, x, monkeypatch, env):
    for k in ("DDA_GJ_ONLY", "DDA_SWEEP_FALLBACK", "DDA_SWEEP_KERNEL"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    with make_problem(s, precond=2, max_rhs=nrhs, precision=fp32) as prob:
        prob.build_preconditioner(0.1)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    for k in env:
        monkeypatch.delenv(k)
    return z


def _box(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 1.0, seed, k=1.0, d=0.25)
    rng = np.random.default_rng(seed)
    s.eps = (2.0 + 0.3 * rng.random(s.mask.shape) + 0.02j).astype(np.complex128)
    return s


@pytest.mark.parametrize("kernel", ["auto", "stream2", "stream", "vector"])
@pytest.mark.parametrize("shape", SHAPES + [(256, 2, 2)])
@pytest.mark.parametrize("fp32", [0, 1])
def test_sweep_matches_gauss_jordan(shape, fp32, kernel, monkeypatch):
    s = _box(shape, 500 + shape[0])
    x = rand_field(shape, 2, 501 + shape[0])
    env = {"DDA_SWEEP_KERNEL": kernel}
    z_sw = _apply(s, 2, fp32, x, monkeypatch, env)
    z_gj = _apply(s, 2, fp32, x, monkeypatch, {"DDA_GJ_ONLY": "1"})
    z_fb = _apply(s, 2, fp32, x, monkeypatch, {"DDA_SWEEP_FALLBACK": "1", **env})
    assert np.array_equal(z_fb, z_gj)
    assert rel_err(z_sw, z_gj) < (2e-6 if fp32 else 1e-12)
    pc = oracle_precond(s, 0.1)
    tol = 1e-5 if fp32 else 1e-10
    for r in range(2):
        assert rel_err(z_sw[r], pc(x[r])) < tol, r
