"""Tile shapes of the x and y FFT passes (rows per tile, columns per tile, tiles per workgroup):
every shape computes each row and column transform by the same arithmetic, so the autotuned and
forced shapes give the launch rule's products bit for bit, and those match the oracle."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, random_waves, rel_err, to_dev
from oracle import fftmatvec, physics

pytestmark = pytest.mark.gpu

# grids whose x / y lengths take the compile-time mixed-radix plans (40, 48, 80, 96) and
# powers of two; "rows,columns,tiles" shapes forced on every pass
CASES = [((12, 20, 16), 3), ((8, 48, 40), 5), ((6, 40, 80), 2), ((4, 96, 32), 4)]
FORCED = ["1,1,1", "2,4,2", "4,8,8"]


def _products(s, nrhs, fp32, seed):
    x = rand_field(s.shape, nrhs, seed)
    dirs, pols = random_waves(nrhs, seed)
    dirs, pols = dirs[:nrhs], pols[:nrhs]
    with make_problem(s, precond=2, max_rhs=nrhs, precision=fp32) as prob:
        prob.build_preconditioner(0.1)
        xd = to_dev(x)
        y = prob.apply_operator(xd, dirs, pols, fp32=bool(fp32)).cpu().numpy()
        z = prob.apply_preconditioner(xd, fp32=bool(fp32)).cpu().numpy()
    return x, dirs, pols, y, z


@pytest.mark.parametrize("shape,nrhs", CASES)
@pytest.mark.parametrize("fp32", [0, 1])
def test_tile_shapes_bit_identical(shape, nrhs, fp32, monkeypatch):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.8, 50 + nx, k=1.1, d=0.3, eps_jitter=0.05)
    monkeypatch.setenv("DDA_FFT_TUNE", "0")
    x, dirs, pols, y0, z0 = _products(s, nrhs, fp32, 60 + nx)
    monkeypatch.delenv("DDA_FFT_TUNE")
    runs = {"tuned": _products(s, nrhs, fp32, 60 + nx)}
    for f in FORCED:
        monkeypatch.setenv("DDA_FFT_FORCE", f)
        runs[f] = _products(s, nrhs, fp32, 60 + nx)
    monkeypatch.delenv("DDA_FFT_FORCE")
    for name, (_, _, _, y, z) in runs.items():
        assert np.array_equal(y, y0), name
        assert np.array_equal(z, z0), name
    # and the rule's products against the oracle
    tol = 1e-5 if fp32 else 1e-10
    pc = oracle_precond(s, 0.1)
    for r in range(nrhs):
        S = physics.lattice_S(dirs[r], pols[r])
        ref = fftmatvec.fft_matvec(x[r], s.mask, s.eps, s.k, s.d, S)
        assert rel_err(y0[r], ref) < tol, r
        assert rel_err(z0[r], pc(x[r])) < tol, r
