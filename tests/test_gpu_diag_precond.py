"""The circulant-plus-diagonal preconditioner P = D + C (Sec. 1, P = D~ + C with the true
diagonal; Sec. 5; option diag_steps) on the GPU through the C-ABI, against the oracle's
fixed-point steps z_{i+1} = Q (v - Delta z_i) around the oracle's circulant blocks."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, rel_err, to_dev
from oracle import circulant, physics, system

pytestmark = pytest.mark.gpu


def _two_material(shape, seed, e2=1.9 + 0.01j, frac=0.6):
    s = w.random_mask(shape[2], shape[1], shape[0], 0.75, seed, k=1.1, d=0.3)
    rng = np.random.default_rng(seed + 500)
    s.eps = np.where(rng.random(s.mask.shape) < frac, 1.7161 + 0.0j, e2).astype(np.complex128)
    return s


def _oracle_plus_diag(s, s_bar, steps, apply_B):
    ati = physics.alpha_tilde_inv(s.eps, s.mask, s.k * s.d, s_bar, "mean_eps")
    delta = circulant.diag_correction(s.eps, s.mask, s.k * s.d, s_bar, ati)
    return lambda v: circulant.apply_plus_diagonal(v, apply_B, delta, steps)


@pytest.mark.parametrize("steps", [1, 3])
@pytest.mark.parametrize("shape,seed,fp32", [((6, 8, 10), 71, 0), ((9, 5, 6), 72, 0),
                                             ((6, 8, 10), 73, 1)])
def test_plus_diagonal_2level_vs_oracle(steps, shape, seed, fp32):
    s = _two_material(shape, seed, e2=3.1684 + 0.05j)
    s_bar = 0.25
    with make_problem(s, precond=2, max_rhs=2, precision=fp32, diag_steps=steps) as prob:
        prob.build_preconditioner(s_bar)
        x = rand_field(shape, 2, seed)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    pc = _oracle_plus_diag(s, s_bar, steps, oracle_precond(s, s_bar))
    for r in range(2):
        assert rel_err(z[r], pc(x[r])) < (1e-5 if fp32 else 1e-10), (steps, r)


def test_plus_diagonal_1level_vs_oracle():
    shape = (4, 5, 12)
    s = _two_material(shape, 74)
    with make_problem(s, precond=1, diag_steps=2) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 1, 74)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    ati = physics.alpha_tilde_inv(s.eps, s.mask, s.k * s.d, 0.0, "mean_eps")
    Dinv = np.linalg.inv(circulant.one_level_blocks(shape, s.k, s.d, ati))
    pc = _oracle_plus_diag(s, 0.0, 2, lambda v: circulant.apply_one_level(v, s.mask, Dinv))
    assert rel_err(z[0], pc(x[0])) < 1e-10


def test_plus_diagonal_homogeneous_is_circulant():
    """For a homogeneous body Delta = 0: every step returns the circulant preconditioner."""
    s = w.random_mask(8, 6, 5, 0.7, 75, k=1.0, d=0.4)
    s.eps = np.full(s.mask.shape, 2.25 + 0.01j)
    x = rand_field(s.shape, 1, 75)
    zs = []
    for steps in (0, 3):
        with make_problem(s, precond=2, diag_steps=steps) as prob:
            prob.build_preconditioner(0.0)
            zs.append(prob.apply_preconditioner(to_dev(x)).cpu().numpy())
    assert rel_err(zs[1], zs[0]) < 1e-13


@pytest.mark.parametrize("axis", [0, 1])
def test_plus_diagonal_in_rotated_frames(axis):
    from test_gpu_dense_axis import _field_from_frame, _field_to_frame, _rotated
    s = _two_material((6, 8, 10), 76)
    with make_problem(s, precond=2, diag_steps=2, dense_axis=axis) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(s.shape, 1, 76)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    sr = _rotated(s, axis)
    pc = _oracle_plus_diag(sr, 0.0, 2, oracle_precond(sr, 0.0))
    ref = _field_from_frame(pc(_field_to_frame(x[0], axis)), axis)
    assert rel_err(z[0], ref) < 1e-10


@pytest.mark.parametrize("solver,side,fp32", [("gmres", "right", 0), ("gmres", "left", 0),
                                              ("gmres", "right", 1), ("bicgstab", "right", 0)])
def test_plus_diagonal_solves_to_dense_lu(solver, side, fp32):
    """Every solver reaches the dense-LU solution with the circulant-plus-diagonal
    preconditioner (in-place applications and scaled Krylov vectors included)."""
    s = _two_material((8, 7, 9), 77, e2=3.1684 + 0.05j)
    dirs, pols = w.plane_wave_z(("x",))
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    with make_problem(s, precond=2, tol=1e-11, diag_steps=2, solver=solver, precond_side=side,
                      precision=fp32) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    assert out["stats"][0]["converged"] == 1
    assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-8
