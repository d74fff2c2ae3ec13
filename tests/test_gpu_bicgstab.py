"""GPU BiCGStab (the paper's second solver, Sec. 4) through the C-ABI vs the CPU oracle."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rel_err, random_waves
from oracle import bicgstab, fftmatvec, physics, system, xsec

pytestmark = pytest.mark.gpu


def _oracle_bicgstab(s, dvec, pvec, precond, tol):
    """The oracle's right-preconditioned BiCGStab on the FFT operator (same P as the GPU's
    build_preconditioner(0): alpha~^{-1} from the mean permittivity)."""
    S = physics.lattice_S(dvec, pvec)
    b = system.incident_field(s.mask, s.k, s.d, dvec, pvec)
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d)
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh)
    pc = oracle_precond(s) if precond else None
    return bicgstab.bicgstab(mv, b, precond=pc, tol=tol, maxit=4000)


@pytest.mark.parametrize("precond", [0, 2])
def test_c1_bicgstab_vs_dense_lu(precond):
    """c1 (16^3 prism, x = 2) solved by GPU BiCGStab at tol 1e-11 against dense LU."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=precond, tol=1e-11, solver="bicgstab", max_iter=4000) as prob:
        if precond:
            prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    st = out["stats"][0]
    assert st["converged"] == 1 and st["rel_residual"] <= 1e-11
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-9
    ce = xsec.c_ext(cref, s.mask, s.k, s.d, dirs[0], pols[0])
    assert abs(out["cext"][0] - ce) < 1e-8 * ce


@pytest.mark.parametrize("precond", [0, 2])
def test_c1_bicgstab_iterations_match_oracle(precond):
    """At the paper's BiCGStab tolerance 1e-5 the GPU takes the oracle's iterations (the
    recurrences agree up to reduction order) and lands on the oracle's iterate."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=precond, tol=1e-5, solver="bicgstab", max_iter=4000) as prob:
        if precond:
            prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    st = out["stats"][0]
    xo, info = _oracle_bicgstab(s, dirs[0], pols[0], precond, 1e-5)
    assert info["converged"] and st["converged"] == 1 and st["rel_residual"] <= 1e-5
    assert abs(st["iters"] - info["iters"]) <= 1, (st["iters"], info["iters"])
    if st["iters"] == info["iters"]:
        assert rel_err(out["c"][0].cpu().numpy(), xo) < 1e-7


def test_c1_bicgstab_precond_beats_plain():
    """The 2-level circulant preconditioner cuts BiCGStab's iterations (Sec. 4)."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    its = {}
    for precond in (0, 2):
        with make_problem(s, precond=precond, tol=1e-5, solver="bicgstab", max_iter=4000) as prob:
            if precond:
                prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
        assert out["stats"][0]["converged"] == 1
        its[precond] = out["stats"][0]["iters"]
    assert its[2] < its[0], its


def test_bicgstab_multi_rhs_batch_matches_single_solves():
    """Three waves with different LDR factors in one block: each RHS runs its own recurrence
    (own scalars, own stopping) and matches its single-RHS solve."""
    s = w.hex_prism_grid(3.0, 0.8, 12, 1.31)
    dirs, pols = random_waves(3, 91)
    dirs, pols = dirs[:3], pols[:3]
    s_bar = float(np.mean(np.sum((dirs * pols) ** 2, axis=1)))
    with make_problem(s, precond=2, tol=1e-10, max_rhs=3, solver="bicgstab") as prob:
        prob.build_preconditioner(s_bar)
        out = prob.solve(dirs, pols)
        c = out["c"].cpu().numpy()
        for r in range(3):
            one = prob.solve(dirs[r:r + 1], pols[r:r + 1])
            assert one["stats"][0]["iters"] == out["stats"][r]["iters"], r
            assert rel_err(c[r], one["c"][0].cpu().numpy()) < 1e-12, r
            assert out["stats"][r]["converged"] == 1
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[1], pols[1]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[1], pols[1])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    assert rel_err(c[1], cref) < 1e-8


def test_bicgstab_cap_warm_start_and_degenerate():
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    with make_problem(s, precond=0, tol=1e-10, max_iter=3, solver="bicgstab") as prob:
        out = prob.solve(dirs, pols)
        assert out["status"] == 1 and out["stats"][0]["converged"] == 0
        assert out["stats"][0]["iters"] == 3
    with make_problem(s, precond=2, tol=1e-10, solver="bicgstab") as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
        out2 = prob.solve(dirs, pols, x0=out["c"])
        assert out2["stats"][0]["iters"] == 0 and out2["status"] == 0
    # a 1 x 1 x n column: the 2-level P is the exact inverse, one step solves it
    s = w.cuboid_grid(1, 1, 9, 2.0, 0.3, 1.31)
    with make_problem(s, precond=2, tol=1e-12, solver="bicgstab") as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    assert out["stats"][0]["iters"] == 1 and out["stats"][0]["converged"] == 1
