"""The dense_axis option (circulant levels on any two axes, Sec. 5): the library works in a
rotated frame, so the operator, solution, cross sections and gradient must not depend on it,
and its preconditioner must be the oracle's 2-level preconditioner of the rotated box."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, random_waves, rel_err, to_dev
from oracle import physics, system

pytestmark = pytest.mark.gpu

AX = {2: (0, 1, 2), 0: (1, 2, 0), 1: (2, 0, 1)}  # internal axis k is the caller's axis AX[k]


def _order(axis):
    ax = AX[axis]
    return (2 - ax[2], 2 - ax[1], 2 - ax[0])  # numpy axes of [nz][ny][nx] -> rotated box


def _box_to_frame(a, axis):
    return np.ascontiguousarray(np.transpose(a, _order(axis)))


def _field_to_frame(x, axis):
    """[3][nz][ny][nx] in the caller's frame -> the rotated frame (components rotate too)."""
    return np.stack([_box_to_frame(x[AX[axis][a]], axis) for a in range(3)])


def _field_from_frame(xi, axis):
    inv = np.argsort(_order(axis))
    out = np.empty((3,) + tuple(xi.shape[1 + i] for i in inv), dtype=xi.dtype)
    for a in range(3):
        out[AX[axis][a]] = np.transpose(xi[a], inv)
    return out


def _rotated(s, axis):
    return w.Scatterer(s.name + f"_ax{axis}", _box_to_frame(s.mask, axis), _box_to_frame(s.eps, axis),
                       k=s.k, d=s.d)


def test_frame_helpers_roundtrip():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 4, 5, 6))
    for axis in (0, 1, 2):
        assert np.array_equal(_field_from_frame(_field_to_frame(x, axis), axis), x)


@pytest.mark.parametrize("axis", [0, 1])
def test_operator_does_not_depend_on_dense_axis(axis):
    s = w.random_mask(10, 8, 6, 0.7, 71, k=1.2, d=0.3, eps_jitter=0.05)
    dirs, pols = random_waves(2, 71)
    x = rand_field(s.shape, 2, 71, s.mask)
    ys = {}
    for ax in (2, axis):
        with make_problem(s, precond=0, max_rhs=2, dense_axis=ax) as prob:
            ys[ax] = prob.apply_operator(to_dev(x), dirs[:2], pols[:2]).cpu().numpy()
    assert rel_err(ys[axis], ys[2]) < 1e-12


@pytest.mark.parametrize("axis,shape,seed", [(0, (6, 8, 10), 72), (1, (7, 6, 8), 73), (0, (5, 9, 4), 74)])
def test_preconditioner_is_the_rotated_boxs(axis, shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.75, seed, k=1.1, d=0.35, eps_jitter=0.05)
    with make_problem(s, precond=2, max_rhs=2, dense_axis=axis) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 2, seed)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    pc = oracle_precond(_rotated(s, axis))
    for r in range(2):
        ref = _field_from_frame(pc(_field_to_frame(x[r], axis)), axis)
        assert rel_err(z[r], ref) < 1e-10, (axis, r)


@pytest.mark.parametrize("axis", [0, 1])
def test_solve_and_gradient_do_not_depend_on_dense_axis(axis):
    s = w.hex_prism_grid(3.0, 2.0, 12, 1.31 + 0.02j)  # elongated along z
    dirs, pols = random_waves(1, 75)
    dirs, pols = dirs[:1], pols[:1]
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    res = {}
    for ax in (2, axis):
        with make_problem(s, precond=2, tol=1e-11, dense_axis=ax) as prob:
            prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
            g, ce, _, _ = prob.grad_cext(dirs[0], pols[0])
        assert out["stats"][0]["converged"] == 1
        assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-9, ax
        res[ax] = (out, g.cpu().numpy(), ce)
    o2, g2, c2 = res[2]
    oa, ga, ca = res[axis]
    for key in ("cext", "cabs", "csca"):
        assert abs(oa[key][0] - o2[key][0]) <= 1e-8 * abs(o2["cext"][0])
    assert abs(ca - c2) <= 1e-8 * abs(c2)
    assert rel_err(ga, g2) < 1e-7
