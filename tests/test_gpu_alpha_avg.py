"""The three readings of the preconditioner's constant diagonal alpha~^{-1} (Sec. 1, Sec. 3.1;
option alpha_avg) on the GPU through the C-ABI, against the oracle's blocks built with the
same alpha~ on inhomogeneous bodies."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, rel_err, to_dev
from oracle import physics, system

pytestmark = pytest.mark.gpu

VARIANTS = ["mean_eps", "mean_alpha", "mode"]


def _two_material(shape, seed, frac=0.65):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.75, seed, k=1.2, d=0.3)
    rng = np.random.default_rng(seed + 1000)
    e1, e2 = 1.7161 + 0.0j, 3.1684 + 0.05j
    s.eps = np.where(rng.random(s.mask.shape) < frac, e1, e2).astype(np.complex128)
    return s


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape,seed,fp32", [((6, 8, 10), 91, 0), ((9, 5, 6), 92, 0),
                                             ((6, 8, 10), 93, 1)])
def test_preconditioner_alpha_variants_vs_oracle(variant, shape, seed, fp32):
    s = _two_material(shape, seed)
    s_bar = 0.25
    with make_problem(s, precond=2, max_rhs=2, precision=fp32, alpha_avg=variant) as prob:
        prob.build_preconditioner(s_bar)
        x = rand_field(shape, 2, seed)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    pc = oracle_precond(s, s_bar, variant)
    for r in range(2):
        assert rel_err(z[r], pc(x[r])) < (1e-5 if fp32 else 1e-10), (variant, r)


def test_alpha_variants_differ_and_solve_to_dense_lu():
    """On a two-material body the three readings give different preconditioners; each one's
    solve reaches the dense-LU solution (the preconditioner changes only the iterations)."""
    s = _two_material((8, 7, 9), 95, frac=0.6)
    dirs, pols = w.plane_wave_z(("x",))
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    atis = {v: physics.alpha_tilde_inv(s.eps, s.mask, s.k * s.d, 0.0, v) for v in VARIANTS}
    assert len({round(a.real, 9) for a in atis.values()}) == 3
    for v in VARIANTS:
        with make_problem(s, precond=2, tol=1e-11, alpha_avg=v) as prob:
            prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
        assert out["stats"][0]["converged"] == 1
        assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-8, v


@pytest.mark.parametrize("variant", ["mean_alpha", "mode"])
def test_one_level_preconditioner_alpha_variants(variant):
    """The 1-level preconditioner (precond = 1) takes the same alpha~ readings."""
    from oracle import circulant
    shape = (4, 5, 12)
    s = _two_material(shape, 97)
    with make_problem(s, precond=1, alpha_avg=variant) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 1, 97)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    ati = physics.alpha_tilde_inv(s.eps, s.mask, s.k * s.d, 0.0, variant)
    Dinv = np.linalg.inv(circulant.one_level_blocks(shape, s.k, s.d, ati))
    assert rel_err(z[0], circulant.apply_one_level(x[0], s.mask, Dinv)) < 1e-10


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("variant", ["mean_alpha", "mode"])
def test_alpha_variants_in_rotated_frames(axis, variant):
    """With another dense axis the library works in a rotated frame; the readings depend on
    the permittivity values only (the mode's tie rule too), so the preconditioner is the
    oracle's for the rotated box with the same alpha~."""
    from test_gpu_dense_axis import _field_from_frame, _field_to_frame, _rotated
    s = _two_material((6, 8, 10), 98, frac=0.5)
    with make_problem(s, precond=2, alpha_avg=variant, dense_axis=axis) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(s.shape, 1, 98)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    pc = oracle_precond(_rotated(s, axis), 0.0, variant)
    ref = _field_from_frame(pc(_field_to_frame(x[0], axis)), axis)
    assert rel_err(z[0], ref) < 1e-10
