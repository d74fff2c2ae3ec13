"""The packed symmetric block product of the 2-level preconditioner (even dense extents) against
the oracle, over tile-row counts ntr = ceil(3 nz / 32) from 1 to 24, odd and even, one to eight
right-hand sides (full and partial chunks of one and two column blocks), both precisions."""


import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _full_box(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 1.0, seed, k=1.0, d=0.25)
    rng = np.random.default_rng(seed)
    s.eps = (2.0 + 0.3 * rng.random(s.mask.shape) + 0.02j).astype(np.complex128)
    return s


# nz even (packed symmetric tiles); tile rows ntr = ceil(3 nz / 32): 1, 2, 3, 7, 9, 12, 16, 24
SHAPES = [(2, 6, 5), (12, 4, 6), (24, 4, 3), (72, 3, 4), (96, 2, 3), (128, 2, 3), (168, 2, 2),
          (256, 2, 3)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("nrhs,fp32", [(1, 0), (2, 0), (2, 1), (3, 0), (5, 1), (8, 0), (8, 1)])
def test_block_product_tile_rows(shape, nrhs, fp32):
    s = _full_box(shape, 300 + shape[0])
    x = rand_field(shape, nrhs, 301 + shape[0])
    with make_problem(s, precond=2, max_rhs=nrhs, precision=fp32) as prob:
        prob.build_preconditioner(0.1)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    pc = oracle_precond(s, 0.1)
    tol = 1e-5 if fp32 else 1e-10
    for r in range(nrhs):
        assert rel_err(z[r], pc(x[r])) < tol, r
