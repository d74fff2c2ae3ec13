"""CPU checks of the C-ABI boundary: the library loads, exports every declared symbol, and
rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dda.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dda_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1903_09802_amd import dda
    return dda.load()


def test_header_declares_the_boundary():
    names = _declared()
    from paper_1903_09802_amd import dda
    assert set(names) == set(dda.EXPORTS), names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options(lib):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    assert (o.restart, o.max_iter, o.tol, o.precond, o.precision, o.max_rhs) == (30, 2000, 1e-5, 2, 0, 1)
    assert o.solver == 0 and o.dense_axis == 2 and o.left_precond == 0 and o.alpha_avg == 0
    assert o.diag_steps == 0 and o.graph == 1


def _struct_fields(name):
    """Field names of ``typedef struct { ... } name;`` in the header, in declaration order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", txt).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            out += [v.strip().lstrip("*") for v in re.sub(r"^[a-z_0-9 ]+?\s(?=\*?[a-z_]+(,|$))", "",
                                                           decl).split(",")]
    return out


def test_binding_structs_mirror_the_header():
    """The ctypes layouts of dda_options and dda_stats follow the header field by field."""
    from paper_1903_09802_amd import dda
    assert _struct_fields("dda_options") == [f for f, _ in dda.Options._fields_]
    assert _struct_fields("dda_stats") == [f for f, _ in dda.Stats._fields_]
    assert "t_setup" in _struct_fields("dda_stats") and "history" in _struct_fields("dda_stats")


def test_lattice_factor(lib):
    """S = sum_j (d_j e_j)^2 per wave (Sec. 2.1) and the batch mean, computed by the library on
    the host; malformed waves are rejected."""
    import numpy as np
    from paper_1903_09802_amd import dda
    d = np.array([[0, 0, 1.0], [1 / np.sqrt(2), 0, 1 / np.sqrt(2)], [1.0, 0, 0]])
    e = np.array([[1.0, 0, 0], [1 / np.sqrt(2), 0, -1 / np.sqrt(2)], [0, 0.6, 0.8]])
    S, mean = dda.lattice_factor(d, e)
    ref = np.sum((d * e) ** 2, axis=1)
    assert np.allclose(S, ref, atol=1e-15) and abs(mean - ref.mean()) < 1e-15
    assert abs(S[1] - 0.5) < 1e-15 and S[0] == 0.0
    with pytest.raises(dda.DDAError) as ei:
        dda.lattice_factor([[0, 0, 1.0]], [[0, 0.6, 0.8]])  # not orthogonal
    assert ei.value.status == -1
    assert lib.dda_lattice_factor(0, None, None, None, None) == -1


@pytest.mark.parametrize("graph", [-1, 2])
def test_create_rejects_bad_graph(lib, graph):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.graph = graph
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"graph" in lib.dda_last_error()


@pytest.mark.parametrize("precond", [-1, 3])
def test_create_rejects_bad_precond(lib, precond):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.precond = precond
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None


@pytest.mark.parametrize("axis", [-1, 3])
def test_create_rejects_bad_dense_axis(lib, axis):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.dense_axis = axis
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None


@pytest.mark.parametrize("left,solver", [(-1, 0), (2, 0), (1, 1)])
def test_create_rejects_bad_left_precond(lib, left, solver):
    """left_precond is 0 or 1, and a GMRES option only."""
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.left_precond, o.solver = left, solver
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"left" in lib.dda_last_error()


@pytest.mark.parametrize("avg", [-1, 3])
def test_create_rejects_bad_alpha_avg(lib, avg):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.alpha_avg = avg
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"alpha_avg" in lib.dda_last_error()


@pytest.mark.parametrize("steps,precond", [(-1, 2), (33, 2), (1, 0)])
def test_create_rejects_bad_diag_steps(lib, steps, precond):
    """diag_steps is in [0, 32] and needs a preconditioner."""
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.diag_steps, o.precond = steps, precond
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"diag_steps" in lib.dda_last_error()


@pytest.mark.parametrize("solver,precision,restart,status", [
    (2, 0, 30, -1),   # unknown solver
    (1, 1, 30, -5),   # BiCGStab has no FP32 mode
    (1, 0, 5, -1),    # BiCGStab's work vectors need restart >= 7
    (0, 0, 0, -1),    # GMRES(m) needs m >= 1
    (0, 0, 1024, -1),  # and at most 1023 basis vectors beyond the first
])
def test_create_rejects_bad_solver_options(lib, solver, precision, restart, status):
    from paper_1903_09802_amd import dda
    o = dda.default_options()
    o.solver, o.precision, o.restart = solver, precision, restart
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: option validation fails first
    st = lib.dda_create(4, 4, 4, dummy, dummy, 1.0, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert st == status
    assert h.value is None


@pytest.mark.parametrize("dims,k,d,status", [
    ((0, 4, 4), 1.0, 0.1, -1),
    ((4, 4, 4), -1.0, 0.1, -1),
    ((4, 4, 4), 1.0, 0.0, -1),
    ((11, 4, 4), 1.0, 0.1, -5),   # 11 is not 7-smooth
    ((4, 4, 1024), 1.0, 0.1, -5),
])
def test_create_rejects_bad_arguments_before_device_work(lib, dims, k, d, status):
    from paper_1903_09802_amd import dda
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    st = lib.dda_create(dims[0], dims[1], dims[2], dummy, dummy, k, d, None, None, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert len(lib.dda_last_error()) > 0


def test_null_handle_calls(lib):
    assert lib.dda_build_preconditioner(None, 0.0) == -1
    assert lib.dda_profile_count(None) == 0
    assert lib.dda_profile_only(None, b"pc_gemv_f64") == -1
    lib.dda_destroy(None)


def test_product_path_fails_loudly_without_library(tmp_path):
    from paper_1903_09802_amd import dda
    with pytest.raises(RuntimeError, match="missing"):
        saved = dda._lib
        dda._lib = None
        try:
            dda.load(str(tmp_path / "nope.so"))
        finally:
            dda._lib = saved
