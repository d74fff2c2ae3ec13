"""The library's per-kernel timing: every kind, or one kind alone (dda_profile_only)."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem

pytestmark = pytest.mark.gpu


def test_profile_every_kind_then_one_kind():
    s = w.hex_prism_grid(3.0, 0.8, 12, 1.31)
    dirs = np.array([[0.0, 0.0, 1.0]])
    pols = np.array([[1.0, 0.0, 0.0]])
    with make_problem(s, precond=2, tol=1e-8, max_rhs=1) as prob:
        prob.profile_enable(True)
        prob.build_preconditioner(0.0)
        ref = prob.solve(dirs, pols, return_c=False)
        every = {k["name"]: k for k in prob.profile() if k["launches"]}
        assert {"pc_gemv_f64", "zpass_f64", "kry_gs_dots"} <= set(every), sorted(every)
        prob.profile_enable(True)  # resets the counts
        prob.profile_only("pc_gemv_f64")
        out = prob.solve(dirs, pols, return_c=False)
        one = {k["name"]: k for k in prob.profile() if k["launches"]}
        assert set(one) == {"pc_gemv_f64"}, sorted(one)
        n1, n0 = one["pc_gemv_f64"]["launches"], every["pc_gemv_f64"]["launches"]
        assert abs(n1 - n0) <= max(2, n0 // 10), (n1, n0)
        assert one["pc_gemv_f64"]["total_ms"] > 0
        # timing changes nothing in the results
        assert out["cext"][0] == ref["cext"][0] and out["stats"][0]["iters"] == ref["stats"][0]["iters"]
        prob.profile_enable(True)
        prob.profile_only(None)
        prob.solve(dirs, pols, return_c=False)
        again = {k["name"] for k in prob.profile() if k["launches"]}
        assert {"pc_gemv_f64", "zpass_f64", "kry_gs_dots", "kry_multiaxpy"} <= again, sorted(again)
