"""GPU GMRES solves, cross sections, refinement, batching and error paths vs the CPU oracle."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, rel_err, random_waves, to_dev, torch_inputs
from oracle import circulant, fftmatvec, gmres, physics, system, xsec

pytestmark = pytest.mark.gpu


def _oracle_solution(s, dvec, pvec, tol=1e-13):
    S = physics.lattice_S(dvec, pvec)
    b = system.incident_field(s.mask, s.k, s.d, dvec, pvec)
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d)
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh)
    c, info = gmres.gmres(mv, b, restart=30, tol=tol, maxit=5000)
    assert info["converged"]
    return c, xsec.cross_sections(c, s.mask, s.eps, s.k, s.d, dvec, pvec)


@pytest.mark.parametrize("precond", [0, 2])
def test_c1_solution_and_cross_sections_vs_oracle(precond):
    """c1 (16^3 prism, x = 2): GPU GMRES(30) at tol 1e-11 vs the oracle's converged solution."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=precond, tol=1e-11) as prob:
        if precond:
            prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    c = out["c"][0].cpu().numpy()
    cref, (ce, ca, cs) = _oracle_solution(s, dirs[0], pols[0])
    assert out["stats"][0]["converged"] == 1
    assert rel_err(c, cref) < 1e-9
    assert abs(out["cext"][0] - ce) < 1e-5 * ce
    assert abs(out["csca"][0] - cs) < 1e-5 * cs
    assert abs(out["cabs"][0]) < 1e-5 * ce  # lossless ice: C_abs vanishes


def test_c1_dense_lu_reference():
    """c1 against dense LU of the 8064-unknown system (the direct definition)."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=2, tol=1e-11) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, 0.0)
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-9
    ce = xsec.c_ext(cref, s.mask, s.k, s.d, dirs[0], pols[0])
    assert abs(out["cext"][0] - ce) < 1e-8 * ce


def test_c1_config_tolerance_precond_beats_plain():
    """At the c1 tolerance 1e-6 both solvers meet the true residual; the circulant
    preconditioner needs fewer iterations (the paper's central claim, Sec. 4)."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    its = {}
    for precond in (0, 2):
        with make_problem(s, precond=precond, tol=1e-6) as prob:
            if precond:
                prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
        st = out["stats"][0]
        assert st["converged"] == 1 and st["rel_residual"] <= 1e-6
        its[precond] = st["iters"]
    assert its[2] < its[0], its


def test_multi_rhs_batch_matches_single_solves():
    """Four waves with different directions (different LDR factors S) in one block."""
    s = w.hex_prism_grid(3.0, 0.8, 12, 1.31)
    dirs, pols = random_waves(4, 77)
    with make_problem(s, precond=2, tol=1e-11, max_rhs=4) as prob:
        prob.build_preconditioner(float(np.mean(np.sum((dirs * pols) ** 2, axis=1))))
        out = prob.solve(dirs, pols)
    c = out["c"].cpu().numpy()
    for r in range(4):
        cref, (ce, ca, cs) = _oracle_solution(s, dirs[r], pols[r])
        assert rel_err(c[r], cref) < 1e-8, r
        assert abs(out["cext"][r] - ce) < 1e-6 * ce
        assert out["stats"][r]["converged"] == 1


@pytest.mark.parametrize("grid,x", [(12, 3.0), (40, 8.0)])
def test_batch_equals_one_wave_solves_bitwise(grid, x):
    """A block of waves reproduces, bit for bit, the same waves solved one per call: every
    per-RHS reduction has a fixed order that does not depend on the block, and a wave's
    iterations do not depend on the others (the batch benchmark's comparison)."""
    s = w.hex_prism_grid(x, 0.8, grid, 1.31)
    dirs, pols = random_waves(6, 78 + grid)
    sbar = float(np.mean(np.sum((dirs * pols) ** 2, axis=1)))
    with make_problem(s, precond=2, tol=1e-5, max_rhs=6) as prob:
        prob.build_preconditioner(sbar)
        out = prob.solve(dirs, pols)
    with make_problem(s, precond=2, tol=1e-5, max_rhs=1) as prob:
        prob.build_preconditioner(sbar)
        singles = [prob.solve(dirs[r:r + 1], pols[r:r + 1]) for r in range(6)]
    c = out["c"].cpu().numpy()
    for r, o in enumerate(singles):
        assert out["stats"][r]["converged"] == 1 and o["stats"][0]["converged"] == 1
        assert out["stats"][r]["iters"] == o["stats"][0]["iters"], r
        assert np.array_equal(c[r], o["c"][0].cpu().numpy()), r
        assert out["cext"][r] == o["cext"][0] and out["csca"][r] == o["csca"][0], r


def test_fp32_refined_batch_matches_fp64_one_wave_solves():
    """The FP32-refined form on a block of waves against the plain FP64 path (one wave per
    solve) at the same tolerance: the same solution to that tolerance."""
    s = w.hex_prism_grid(6.0, 1.0, 24, 1.31)
    dirs, pols = random_waves(8, 91)
    sbar = float(np.mean(np.sum((dirs * pols) ** 2, axis=1)))
    tol = 1e-8
    with make_problem(s, precond=2, tol=tol, max_rhs=8, precision=1) as prob:
        prob.build_preconditioner(sbar)
        out = prob.solve(dirs, pols)
    with make_problem(s, precond=2, tol=tol, max_rhs=1) as prob:
        prob.build_preconditioner(sbar)
        singles = [prob.solve(dirs[r:r + 1], pols[r:r + 1]) for r in range(8)]
    c = out["c"].cpu().numpy()
    for r, o in enumerate(singles):
        assert out["stats"][r]["converged"] == 1 and o["stats"][0]["converged"] == 1
        assert out["stats"][r]["rel_residual"] <= tol
        # both solutions are within the system's conditioning of the exact one
        assert rel_err(c[r], o["c"][0].cpu().numpy()) < 1e-5, r
        assert abs(out["cext"][r] - o["cext"][0]) < 1e-6 * abs(o["cext"][0]), r
        assert abs(out["csca"][r] - o["csca"][0]) < 1e-6 * abs(o["csca"][0]), r


def test_optical_theorem_on_gpu_lossy():
    s = w.hex_prism_grid(4.0, 1.0, 16, 1.31 + 0.05j)
    dirs, pols = w.plane_wave_z(("y",))
    with make_problem(s, precond=2, tol=1e-10) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    ce, ca, cs = out["cext"][0], out["cabs"][0], out["csca"][0]
    assert ca > 0 and abs(ce - ca - cs) < 1e-7 * ce


def test_refinement_fp32_matches_fp64():
    """FP32 operator + preconditioner inside FP64 refinement reaches the FP64 answer."""
    s = w.hex_prism_grid(4.0, 2.0, 16, 1.31 + 0.001j)
    dirs, pols = w.plane_wave_z(("x",))
    res = {}
    for precision in (0, 1):
        with make_problem(s, precond=2, tol=1e-8, precision=precision) as prob:
            prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
        st = out["stats"][0]
        assert st["converged"] == 1 and st["rel_residual"] <= 1e-8
        if precision:
            assert st["refinements"] >= 1
        res[precision] = out
    c0, c1 = res[0]["c"].cpu().numpy(), res[1]["c"].cpu().numpy()
    assert rel_err(c1, c0) < 1e-6
    for key in ("cext", "csca"):
        assert abs(res[1][key][0] - res[0][key][0]) < 1e-6 * res[0][key][0]


def test_warm_start_and_not_converged_status():
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    with make_problem(s, precond=0, tol=1e-10, max_iter=3) as prob:
        out = prob.solve(dirs, pols)
        assert out["status"] == 1 and out["stats"][0]["converged"] == 0
        assert out["stats"][0]["iters"] == 3
    with make_problem(s, precond=0, tol=1e-10) as prob:
        out = prob.solve(dirs, pols)
        out2 = prob.solve(dirs, pols, x0=out["c"])
        assert out2["stats"][0]["iters"] == 0 and out2["status"] == 0


def test_error_paths():
    import torch
    from paper_1903_09802_amd.dda import DDAError, Problem
    s = w.hex_prism_grid(2.0, 1.0, 8, 1.31)
    m, e = torch_inputs(s)
    e_bad = e.clone()
    occ = np.flatnonzero(s.mask.ravel())
    e_bad.view(-1)[int(occ[3])] = 1.0
    with pytest.raises(DDAError) as ei:
        Problem(m, e_bad, s.k, s.d)
    assert ei.value.status == -1
    with pytest.raises(DDAError) as ei:
        Problem(torch.zeros_like(m), e, s.k, s.d)
    assert ei.value.status == -1
    prob = Problem(m, e, s.k, s.d, precond=2)
    dirs, pols = w.plane_wave_z(("x",))
    with pytest.raises(DDAError) as ei:
        prob.solve(dirs, pols)  # preconditioner not built
    assert ei.value.status == -4
    with pytest.raises(DDAError) as ei:
        prob.solve(np.array([[0, 0, 1.0]]), np.array([[0, 0.6, 0.8]]))  # not orthogonal
    assert ei.value.status == -1
    with pytest.raises(DDAError) as ei:
        prob.solve(np.tile(dirs, (2, 1)), np.tile(pols, (2, 1)))  # nrhs > max_rhs
    assert ei.value.status == -1
    prob.close()


def test_degenerate_grids_solve():
    """A single voxel (c = alpha E0) and a 1 x 1 x n column (2-level P is exact: one iteration)."""
    s = w.cuboid_grid(1, 1, 1, 1.0, 0.25, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    with make_problem(s, precond=2, tol=1e-12) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    alpha = 1.0 / physics.alpha_inv(1.31 ** 2, 0.25, 0.0)
    assert abs(out["c"][0, 0, 0, 0, 0].item() - alpha) < 1e-14
    s = w.cuboid_grid(1, 1, 9, 2.0, 0.3, 1.31)
    with make_problem(s, precond=2, tol=1e-12) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols)
    assert out["stats"][0]["iters"] == 1 and out["stats"][0]["converged"] == 1
