"""The allocation-free cross sections (dda_cross_sections_noalloc) against dda_cross_sections
through the C-ABI: two calls in a row, the second on a smaller problem with fewer waves, both
to the oracle's tolerance for reductions in another order; more waves than the static scratch
holds are refused."""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, rand_field, random_waves, to_dev

pytestmark = pytest.mark.gpu


def _check(s, nwaves, seed, dense_axis=2):
    dirs, pols = random_waves(nwaves, seed)
    dirs, pols = dirs[:nwaves], pols[:nwaves]
    c = to_dev(rand_field(s.shape, nwaves, seed, s.mask))
    with make_problem(s, precond=0, max_rhs=nwaves, dense_axis=dense_axis) as prob:
        ce, ca, _ = prob.cross_sections(c, dirs, pols)
        ce2, ca2 = prob.cross_sections_noalloc(c, dirs, pols)
    assert np.all(np.abs(ca) > 0)
    np.testing.assert_allclose(ce2, ce, rtol=1e-12, atol=1e-14 * np.abs(ce).max())
    np.testing.assert_allclose(ca2, ca, rtol=1e-12, atol=1e-14 * np.abs(ca).max())


def test_noalloc_cross_sections_two_calls_then_smaller():
    big = w.hex_prism_grid(4.0, 1.2, 20, 1.31 + 0.03j)
    _check(big, 5, 71)
    small = w.random_mask(6, 5, 7, 0.7, 72, k=1.3, d=0.3, eps_mean=2.0 + 0.1j, eps_jitter=0.05)
    _check(small, 2, 73)
    _check(small, 3, 74, dense_axis=0)  # a rotated frame


def test_noalloc_cross_sections_limits():
    from paper_1903_09802_amd.dda import DDAError
    s = w.random_mask(6, 5, 4, 0.8, 75, k=1.3, d=0.3)
    dirs, pols = random_waves(17, 75)
    dirs, pols = dirs[:17], pols[:17]
    c = to_dev(rand_field(s.shape, 17, 75, s.mask))
    with make_problem(s, precond=0, max_rhs=17) as prob:
        with pytest.raises(DDAError) as ei:
            prob.cross_sections_noalloc(c, dirs, pols)
        assert ei.value.status == -1 and "16" in str(ei.value)
        ce, ca = prob.cross_sections_noalloc(c[:16], dirs[:16], pols[:16])
        ce_ref, ca_ref, _ = prob.cross_sections(c[:16], dirs[:16], pols[:16])
        np.testing.assert_allclose(ce, ce_ref, rtol=1e-12, atol=1e-14 * np.abs(ce_ref).max())
