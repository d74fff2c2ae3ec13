"""Restart cycles decided on the device: HIP-graph replays against the same kernels launched one
by one, the per-step residual history against the oracle's GMRES, early stops inside a cycle,
graphs dropped when the preconditioner is rebuilt, and the timing fields of dda_stats."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rel_err, random_waves
from oracle import fftmatvec, gmres, physics, system

pytestmark = pytest.mark.gpu


def _solve(s, dirs, pols, graph, **kw):
    with make_problem(s, graph=graph, **kw) as prob:
        if kw.get("precond", 2):
            prob.build_preconditioner(float(np.mean(np.sum((dirs * pols) ** 2, axis=1))))
        return prob.solve(dirs, pols, history=True)


@pytest.mark.parametrize("precond,precision,side", [(2, 0, "right"), (0, 0, "right"), (2, 1, "right"),
                                                    (2, 0, "left"), (1, 0, "right")])
def test_graph_cycles_match_eager_bit_for_bit(precond, precision, side):
    """The captured cycle replays exactly the kernels the eager path launches: same iterates,
    same step counts, same histories; 3 right-hand sides that stop at different steps."""
    s = w.hex_prism_grid(3.0, 1.3, 12, 1.31 + 0.01j)
    dirs, pols = random_waves(3, 909)
    dirs, pols = dirs[:3], pols[:3]
    kw = dict(precond=precond, precision=precision, precond_side=side, tol=1e-9, restart=8,
              max_rhs=3)
    eager = _solve(s, dirs, pols, False, **kw)
    graph = _solve(s, dirs, pols, True, **kw)
    for r in range(3):
        ge, gg = eager["stats"][r], graph["stats"][r]
        assert ge["converged"] == gg["converged"] == 1
        assert ge["iters"] == gg["iters"] and ge["cycles"] == gg["cycles"] >= 2
        assert np.array_equal(ge["history"], gg["history"])
        assert ge["rel_residual"] == gg["rel_residual"]
    assert np.array_equal(eager["c"].cpu().numpy(), graph["c"].cpu().numpy())


def test_graph_replays_with_eager_work_between():
    """Several solves on one handle replay the same captured cycles; eager launches (operator
    applications) run between them; every replay matches the first solve and dense LU."""
    import torch
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = random_waves(2, 910)
    dirs, pols = dirs[:2], pols[:2]
    A = [system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[r], pols[r]))
         for r in range(2)]
    b = [system.incident_field(s.mask, s.k, s.d, dirs[r], pols[r]) for r in range(2)]
    cref = [system.compact_to_box(np.linalg.solve(A[r], system.box_to_compact(b[r], s.mask)), s.mask)
            for r in range(2)]
    with make_problem(s, precond=2, tol=1e-11, restart=10, max_rhs=2) as prob:
        prob.build_preconditioner(0.0)
        first = prob.solve(dirs, pols)
        x = torch.randn((2, 3) + s.shape, dtype=torch.complex128, device="cuda")
        for rep in range(4):
            prob.apply_operator(x, dirs, pols)  # eager work between the replays
            torch.cuda.synchronize()
            out = prob.solve(dirs, pols)
            assert np.array_equal(out["c"].cpu().numpy(), first["c"].cpu().numpy()), rep
            assert [st["iters"] for st in out["stats"]] == [st["iters"] for st in first["stats"]]
            for r in range(2):
                assert rel_err(out["c"][r].cpu().numpy(), cref[r]) < 1e-9, (rep, r)
        # one wave, then two again: a second captured configuration beside the first
        one = prob.solve(dirs[:1], pols[:1])
        assert rel_err(one["c"][0].cpu().numpy(), cref[0]) < 1e-9
        again = prob.solve(dirs, pols)
        assert np.array_equal(again["c"].cpu().numpy(), first["c"].cpu().numpy())


def test_history_matches_oracle_gmres():
    """c1 prism, plain GMRES(30) to 1e-6: the per-step residual estimates agree with the oracle's
    textbook GMRES (same Krylov process, different orthogonalisation rounding), are
    non-increasing within each cycle, and the last one is at most the tolerance."""
    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=0, tol=1e-6, restart=30) as prob:
        out = prob.solve(dirs, pols, history=True)
    st = out["stats"][0]
    h = st["history"]
    assert st["history_len"] == st["iters"] == len(h)
    S = physics.lattice_S(dirs[0], pols[0])
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d)
    _, info = gmres.gmres(lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh),
                          b, restart=30, tol=1e-6)
    ho = np.array(info["history"])
    assert abs(len(ho) - len(h)) <= 1
    n = min(len(ho), len(h), 30)
    assert np.max(np.abs(h[:n] - ho[:n]) / ho[:n]) < 1e-6
    for c0 in range(0, len(h), 30):
        seg = h[c0:c0 + 30]
        assert np.all(np.diff(seg) <= 1e-12 * seg[:-1])
    assert h[-1] <= 1e-6


def test_stop_inside_a_cycle_and_rebuild():
    """A right-hand side that converges mid-cycle stops there (the cycle's remaining segments of
    steps are not launched, and the rest of the current one does no work); rebuilding the
    preconditioner drops the captured cycles, and the next solve runs with the new blocks."""
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    with make_problem(s, precond=2, tol=1e-6, restart=200) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols, history=True)
        st = out["stats"][0]
        assert st["cycles"] <= 2 and st["iters"] < 200 and st["converged"] == 1
        assert st["history"][-1] <= 1e-6
        c1 = out["c"][0].cpu().numpy()
        prob.build_preconditioner(0.5)  # another diagonal: another preconditioner, same answer
        out2 = prob.solve(dirs, pols)
        assert out2["stats"][0]["converged"] == 1
        assert rel_err(out2["c"][0].cpu().numpy(), c1) < 1e-5
    S = physics.lattice_S(dirs[0], pols[0])
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    pc = oracle_precond(s)
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d)
    _, info = gmres.gmres(lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh),
                          b, precond=pc, restart=200, tol=1e-6)
    assert abs(info["iters"] - st["iters"]) <= 1


def test_stats_timings_and_iteration_cap():
    s = w.hex_prism_grid(3.0, 1.0, 12, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    with make_problem(s, precond=2, tol=1e-12, max_iter=7, restart=5) as prob:
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols, history=True)
    st = out["stats"][0]
    assert out["status"] == 1 and st["converged"] == 0
    assert st["iters"] == 7 and st["cycles"] == 2 and st["history_len"] == 7
    assert st["t_setup"] > 0 and st["t_build"] > 0 and st["t_solve"] > 0
    with make_problem(s, precond=0, tol=1e-6) as prob:
        out = prob.solve(dirs, pols)
    assert out["stats"][0]["t_build"] == 0.0
