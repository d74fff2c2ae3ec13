"""Left-preconditioned GMRES (the paper's P^{-1} A x = P^{-1} b, Sec. 1 eq. general_prec) on
the GPU through the C-ABI, against the oracle's left-preconditioned GMRES and dense LU."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rel_err, random_waves
from oracle import fftmatvec, gmres, physics, system

pytestmark = pytest.mark.gpu


def _system(s, dvec, pvec):
    S = physics.lattice_S(dvec, pvec)
    b = system.incident_field(s.mask, s.k, s.d, dvec, pvec)
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d)
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh)
    return S, b, mv


@pytest.mark.parametrize("restart", [30, 200])
def test_c1_left_gmres_iterations_and_residual_match_oracle(restart):
    """At the paper's tolerance 1e-5 the GPU's left-preconditioned GMRES takes the oracle's
    iterations (up to reduction order) and stops on the preconditioned residual, while the
    reported residual is the true one."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=2, tol=1e-5, restart=restart, precond_side="left") as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    st = out["stats"][0]
    S, b, mv = _system(s, dirs[0], pols[0])
    pc = oracle_precond(s)
    xo, info = gmres.gmres(mv, b, precond=pc, restart=restart, tol=1e-5, side="left")
    assert info["converged"] and st["converged"] == 1
    assert abs(st["iters"] - info["iters"]) <= 1, (st["iters"], info["iters"])
    x = out["c"][0].cpu().numpy()
    prel = np.linalg.norm(pc(b - mv(x))) / np.linalg.norm(pc(b))
    assert prel <= 1e-5 * 1.001
    true = np.linalg.norm(b - mv(x)) / np.linalg.norm(b)
    assert abs(st["rel_residual"] - true) < 1e-3 * true
    if st["iters"] == info["iters"]:
        assert rel_err(x, xo) < 1e-7


@pytest.mark.parametrize("precision", [0, 1])
def test_left_gmres_converges_to_dense_lu(precision):
    """A multi-RHS left-preconditioned solve to tol 1e-11 (FP64, and FP32 cycles inside FP64
    refinement) reaches the dense-LU solution."""
    s = w.hex_prism_grid(3.0, 0.8, 12, 1.31)
    dirs, pols = random_waves(2, 17)
    with make_problem(s, precond=2, tol=1e-11, restart=20, max_rhs=2, precision=precision,
                      precond_side="left") as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs[:2], pols[:2])
    for r in range(2):
        st = out["stats"][r]
        assert st["converged"] == 1 and st["rel_residual"] < 1e-9, st
        A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[r], pols[r]))
        b = system.incident_field(s.mask, s.k, s.d, dirs[r], pols[r])
        cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
        assert rel_err(out["c"][r].cpu().numpy(), cref) < 1e-8


def test_left_side_without_preconditioner_is_plain_gmres():
    """precond = 0 ignores the side: the same iterations and iterate as the default."""
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    res = {}
    for side in ("right", "left"):
        with make_problem(s, precond=0, tol=1e-6, precond_side=side) as prob:
            out = prob.solve(dirs, pols)
        res[side] = (out["stats"][0]["iters"], out["c"][0].cpu().numpy())
    assert res["right"][0] == res["left"][0]
    assert rel_err(res["left"][1], res["right"][1]) == 0.0
