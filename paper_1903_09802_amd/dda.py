"""ctypes binding of ``lib/libdda.so`` (include/dda.h), with torch tensors for device memory.

Argument marshalling only: every step of the solve runs in the HIP library.  Loading fails
loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libdda.so")

OK, NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE",
                -4: "ESTATE", -5: "EUNSUPPORTED"}

# every symbol declared in include/dda.h
EXPORTS = (
    "dda_default_options", "dda_last_error", "dda_lattice_factor", "dda_create",
    "dda_build_preconditioner",
    "dda_solve", "dda_apply_operator", "dda_apply_preconditioner", "dda_cross_sections",
    "dda_cross_sections_noalloc",
    "dda_grad_cext", "dda_destroy", "dda_profile_enable", "dda_profile_only", "dda_profile_count",
    "dda_profile_get",
)


class DDAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iter", ctypes.c_int), ("tol", ctypes.c_double),
                ("precond", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_rhs", ctypes.c_int), ("solver", ctypes.c_int), ("dense_axis", ctypes.c_int),
                ("left_precond", ctypes.c_int), ("alpha_avg", ctypes.c_int),
                ("diag_steps", ctypes.c_int), ("graph", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("cycles", ctypes.c_int), ("refinements", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_build", ctypes.c_double),
                ("t_solve", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_cap", ctypes.c_int), ("history_len", ctypes.c_int)]

    def as_dict(self, history=None):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("history", "history_cap")}
        if history is not None:
            d["history"] = history[:self.history_len].copy()
        return d


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(path)
    vp, dp, ip, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int
    L.dda_default_options.argtypes = [ctypes.POINTER(Options)]
    L.dda_default_options.restype = None
    L.dda_last_error.argtypes = []
    L.dda_last_error.restype = ctypes.c_char_p
    L.dda_lattice_factor.argtypes = [i, dp, dp, dp, dp]
    L.dda_lattice_factor.restype = ip
    L.dda_create.argtypes = [i, i, i, vp, vp, ctypes.c_double, ctypes.c_double,
                             ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    L.dda_create.restype = ip
    L.dda_build_preconditioner.argtypes = [vp, ctypes.c_double]
    L.dda_build_preconditioner.restype = ip
    L.dda_solve.argtypes = [vp, i, dp, dp, vp, vp, dp, dp, dp, ctypes.POINTER(Stats)]
    L.dda_solve.restype = ip
    L.dda_apply_operator.argtypes = [vp, i, dp, dp, vp, vp, i]
    L.dda_apply_operator.restype = ip
    L.dda_apply_preconditioner.argtypes = [vp, i, vp, vp, i]
    L.dda_apply_preconditioner.restype = ip
    L.dda_cross_sections.argtypes = [vp, i, dp, dp, vp, dp, dp, dp]
    L.dda_cross_sections.restype = ip
    L.dda_cross_sections_noalloc.argtypes = [vp, i, dp, dp, vp, dp, dp]
    L.dda_cross_sections_noalloc.restype = ip
    L.dda_grad_cext.argtypes = [vp, dp, dp, vp, dp, ctypes.POINTER(Stats)]
    L.dda_grad_cext.restype = ip
    L.dda_destroy.argtypes = [vp]
    L.dda_destroy.restype = None
    L.dda_profile_enable.argtypes = [vp, i]
    L.dda_profile_enable.restype = ip
    L.dda_profile_only.argtypes = [vp, ctypes.c_char_p]
    L.dda_profile_only.restype = ip
    L.dda_profile_count.argtypes = [vp]
    L.dda_profile_count.restype = ip
    L.dda_profile_get.argtypes = [vp, i, ctypes.POINTER(ctypes.c_char_p),
                                  ctypes.POINTER(ctypes.c_longlong), dp, dp]
    L.dda_profile_get.restype = ip
    _lib = L
    return L


def _check(st: int, allow_not_converged: bool = True):
    if st == OK or (st == NOT_CONVERGED and allow_not_converged):
        return st
    raise DDAError(st, load().dda_last_error().decode())


def default_options() -> Options:
    o = Options()
    load().dda_default_options(ctypes.byref(o))
    return o


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _waves(dirs, pols):
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
    p = np.ascontiguousarray(np.asarray(pols, dtype=np.float64).reshape(-1, 3))
    if d.shape != p.shape:
        raise ValueError("dirs and pols must have the same number of waves")
    return d, p


def lattice_factor(dirs, pols):
    """Per-wave LDR lattice factors S (Sec. 2.1) and their mean, from ``dda_lattice_factor``."""
    d, p = _waves(dirs, pols)
    S = np.zeros(d.shape[0])
    mean = np.zeros(1)
    _check(load().dda_lattice_factor(d.shape[0], _dptr(d), _dptr(p), _dptr(S), _dptr(mean)), False)
    return S, float(mean[0])


def _stats_array(n, history_cap):
    st = (Stats * n)()
    bufs = []
    for r in range(n):
        if history_cap > 0:
            h = np.zeros(history_cap)
            st[r].history = _dptr(h)
            st[r].history_cap = history_cap
            bufs.append(h)
        else:
            bufs.append(None)
    return st, bufs


def _dev(t, dtype):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """One voxelised scatterer on the GPU (handle of ``dda_create``)."""

    def __init__(self, mask, eps, k: float, d: float, *, restart=30, max_iter=2000, tol=1e-5,
                 precond=2, precision=0, max_rhs=1, solver="gmres", dense_axis=2,
                 precond_side="right", alpha_avg="mean_eps", diag_steps=0, graph=True,
                 stream=None):
        import torch
        L = load()
        self.mask = mask.to(device="cuda", dtype=torch.uint8).contiguous()
        self.eps = eps.to(device="cuda", dtype=torch.complex128).contiguous()
        nz, ny, nx = self.mask.shape
        self.shape = (nz, ny, nx)
        self.k, self.d = float(k), float(d)
        o = default_options()
        o.restart, o.max_iter, o.tol = restart, max_iter, tol
        o.precond, o.precision, o.max_rhs = precond, precision, max_rhs
        o.graph = int(bool(graph))
        solvers = {"gmres": 0, "bicgstab": 1}
        if solver not in solvers:
            raise ValueError(f"solver must be one of {sorted(solvers)}")
        o.solver = solvers[solver]
        o.dense_axis = int(dense_axis)
        sides = {"right": 0, "left": 1}
        if precond_side not in sides:
            raise ValueError(f"precond_side must be one of {sorted(sides)}")
        o.left_precond = sides[precond_side]
        avgs = {"mean_eps": 0, "mean_alpha": 1, "mode": 2}
        if alpha_avg not in avgs:
            raise ValueError(f"alpha_avg must be one of {sorted(avgs)}")
        o.alpha_avg = avgs[alpha_avg]
        o.diag_steps = int(diag_steps)
        self.opts = o
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        _check(L.dda_create(nx, ny, nz, _dev(self.mask, torch.uint8), _dev(self.eps, torch.complex128),
                            self.k, self.d, ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream),
                            ctypes.byref(h)), False)
        self.h = h

    # -- lifetime
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().dda_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls
    def build_preconditioner(self, s_bar: float = 0.0):
        _check(load().dda_build_preconditioner(self.h, float(s_bar)), False)

    def field_shape(self, nrhs):
        return (nrhs, 3) + self.shape

    def solve(self, dirs, pols, x0=None, return_c=True, xsec=True, history=False):
        """Solve for the waves (dirs, pols); with history=True each stats entry carries the
        residual after every iteration (``history``)."""
        import torch
        d, p = _waves(dirs, pols)
        n = d.shape[0]
        c = torch.empty(self.field_shape(n), dtype=torch.complex128, device="cuda") if return_c else None
        ce, ca, cs = (np.zeros(n) for _ in range(3))
        st, bufs = _stats_array(n, self.opts.max_iter if history else 0)
        x0p = _dev(x0, torch.complex128) if x0 is not None else None
        status = _check(load().dda_solve(
            self.h, n, _dptr(d), _dptr(p), x0p, _dev(c, torch.complex128) if c is not None else None,
            _dptr(ce) if xsec else None, _dptr(ca) if xsec else None, _dptr(cs) if xsec else None, st))
        out = dict(status=status, stats=[s.as_dict(b) for s, b in zip(st, bufs)])
        if return_c:
            out["c"] = c
        if xsec:
            out.update(cext=ce, cabs=ca, csca=cs)
        return out

    def apply_operator(self, x, dirs, pols, fp32=False, out=None):
        import torch
        d, p = _waves(dirs, pols)
        y = torch.empty_like(x) if out is None else out
        _check(load().dda_apply_operator(self.h, d.shape[0], _dptr(d), _dptr(p),
                                         _dev(x, torch.complex128), _dev(y, torch.complex128),
                                         int(bool(fp32))), False)
        return y

    def apply_preconditioner(self, x, fp32=False, out=None):
        import torch
        y = torch.empty_like(x) if out is None else out
        _check(load().dda_apply_preconditioner(self.h, x.shape[0], _dev(x, torch.complex128),
                                               _dev(y, torch.complex128), int(bool(fp32))), False)
        return y

    def cross_sections(self, c, dirs, pols):
        import torch
        d, p = _waves(dirs, pols)
        n = d.shape[0]
        ce, ca, cs = (np.zeros(n) for _ in range(3))
        _check(load().dda_cross_sections(self.h, n, _dptr(d), _dptr(p), _dev(c, torch.complex128),
                                         _dptr(ce), _dptr(ca), _dptr(cs)), False)
        return ce, ca, cs

    def cross_sections_noalloc(self, c, dirs, pols):
        """C_ext and C_abs through the allocation-free entry point (at most 16 waves)."""
        import torch
        d, p = _waves(dirs, pols)
        n = d.shape[0]
        ce, ca = np.zeros(n), np.zeros(n)
        _check(load().dda_cross_sections_noalloc(self.h, n, _dptr(d), _dptr(p),
                                                 _dev(c, torch.complex128), _dptr(ce), _dptr(ca)),
               False)
        return ce, ca

    def grad_cext(self, direction, polarisation):
        import torch
        d, p = _waves(direction, polarisation)
        g = torch.empty(self.shape, dtype=torch.complex128, device="cuda")
        ce = np.zeros(1)
        st, _ = _stats_array(2, 0)
        status = _check(load().dda_grad_cext(self.h, _dptr(d), _dptr(p), _dev(g, torch.complex128),
                                             _dptr(ce), st))
        return g, float(ce[0]), [s.as_dict() for s in st], status

    def profile_enable(self, on=True):
        _check(load().dda_profile_enable(self.h, int(bool(on))), False)

    def profile_only(self, name=None):
        """Time only launches of kernel kind ``name`` (None: every kind)."""
        _check(load().dda_profile_only(self.h, name.encode() if name else None), False)

    def profile(self):
        L = load()
        out = []
        for i in range(L.dda_profile_count(self.h)):
            nm = ctypes.c_char_p()
            nl = ctypes.c_longlong()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            _check(L.dda_profile_get(self.h, i, ctypes.byref(nm), ctypes.byref(nl), ctypes.byref(ms),
                                     ctypes.byref(by)), False)
            out.append(dict(name=nm.value.decode(), launches=nl.value, total_ms=ms.value,
                            bytes_per_launch=by.value))
        return out
