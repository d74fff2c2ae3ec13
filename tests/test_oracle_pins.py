"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle through a route other than its own formula:
textbook limits, invariants, numerical differentiation, brute force on tiny
inputs, independent quadratures, and the values the paper prints (Tables 3-4).
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as w
from oracle import adjoint, circulant, fftmatvec, gmres, physics, rows, system, xsec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- polarisability

def test_alpha_matches_ratio_form_of_ldr():
    """1/alpha from the oracle equals the reciprocal of the paper's ratio form
    alpha^LDR = alpha^CM / (1 + alpha^CM [...]) (Sec. 2.1), for complex eps and S."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        eps = 1.0 + 3.0 * rng.random() + 0.3j * rng.random()
        kd = 0.05 + 0.6 * rng.random()
        S = rng.random()
        a_cm = 3.0 / (4.0 * math.pi) * (eps - 1.0) / (eps + 2.0)
        brk = (-1.891531 + eps * 0.1648469 + eps * (-1.7700004) * S) * kd ** 2 - 2j / 3.0 * kd ** 3
        a_ldr = a_cm / (1.0 + a_cm * brk)
        assert abs(physics.alpha_inv(eps, kd, S) * a_ldr - 1.0) < 1e-13


def test_alpha_limits_and_radiative_reaction():
    """kd -> 0 gives Clausius-Mossotti; for real eps, Im(1/alpha) = -(2/3)(kd)^3 exactly
    (the radiative-reaction term, so a lossless dipole absorbs nothing)."""
    eps = 1.7161
    cm = 3.0 / (4.0 * math.pi) * (eps - 1.0) / (eps + 2.0)
    assert abs(1.0 / physics.alpha_inv(eps, 1e-9, 0.0) - cm) < 1e-14
    for kd in (0.1, 0.25, 0.625):
        ai = physics.alpha_inv(eps, kd, 0.3)
        assert abs(ai.imag + 2.0 / 3.0 * kd ** 3) < 1e-15


def test_alpha_derivative_by_finite_differences():
    eps, kd, S = 2.1 + 0.2j, 0.3, 0.4
    h = 1e-6
    fd = (physics.alpha_inv(eps + h, kd, S) - physics.alpha_inv(eps - h, kd, S)) / (2 * h)
    fdi = (physics.alpha_inv(eps + 1j * h, kd, S) - physics.alpha_inv(eps - 1j * h, kd, S)) / (2j * h)
    an = physics.dalpha_inv_deps(eps, kd, S)
    assert abs(fd - an) < 1e-7 * abs(an) and abs(fdi - an) < 1e-7 * abs(an)


def test_lattice_S():
    assert physics.lattice_S((0, 0, 1), (1, 0, 0)) == 0.0
    d = np.array([1.0, 1.0, 1.0]) / math.sqrt(3)
    e = np.array([1.0, -1.0, 0.0]) / math.sqrt(2)
    assert abs(physics.lattice_S(d, e) - 1.0 / 3.0) < 1e-15


# --------------------------------------------------------------------------- Green tensor

def _scalar_green(R, k):
    r = np.linalg.norm(R)
    return np.exp(1j * k * r) / r


@pytest.mark.parametrize("R", [(0.7, -0.3, 0.45), (1.3, 0.2, -2.1), (0.0, 0.9, 0.0)])
def test_green_equals_k2_plus_graddiv_of_scalar(R):
    """G = (k^2 I + grad grad) e^{ikr}/r (Sec. 2), by 4th-order finite differences."""
    k = 1.7
    R = np.array(R)
    h = 1e-3
    eye = np.eye(3)
    H = np.zeros((3, 3), dtype=complex)

    def f(dv):
        return _scalar_green(R + dv, k)

    for a in range(3):
        for b in range(3):
            ea, eb = eye[a] * h, eye[b] * h
            if a == b:
                H[a, a] = (-f(2 * ea) + 16 * f(ea) - 30 * f(0 * ea) + 16 * f(-ea) - f(-2 * ea)) / (12 * h * h)
            else:
                H[a, b] = (f(ea + eb) - f(ea - eb) - f(-ea + eb) + f(-ea - eb)) / (4 * h * h)
    ref = k * k * _scalar_green(R, k) * eye + H
    G = physics.green(R, k)
    assert np.abs(G - ref).max() < 2e-6 * np.abs(ref).max()


def test_green_symmetry_and_table1_parity():
    """G_ab = G_ba, G(-R) = G(R), and the per-axis parity of each of the six blocks
    (Table 1, with the G_yz level-3 entry corrected to odd: g_yz is odd in z)."""
    k = 1.1
    rng = np.random.default_rng(2)
    R = rng.normal(size=(50, 3))
    G = physics.green(R, k)
    assert np.abs(G - np.swapaxes(G, -1, -2)).max() < 1e-14
    assert np.abs(G - physics.green(-R, k)).max() < 1e-14
    # expected parity per (component, axis): odd iff exactly one of a, b equals the axis
    table1 = {  # (+) symmetric / (-) antisymmetric per level x, y, z
        (0, 0): "+++", (0, 1): "--+", (0, 2): "-+-",
        (1, 1): "+++", (1, 2): "+--", (2, 2): "+++",
    }
    for (a, b), pat in table1.items():
        for axis in range(3):
            Rf = R.copy()
            Rf[:, axis] *= -1
            ratio = physics.green(Rf, k)[:, a, b] / G[:, a, b]
            sign = 1.0 if pat[axis] == "+" else -1.0
            assert np.abs(ratio - sign).max() < 1e-12


def test_green_far_field_is_transverse():
    k = 2.0
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    r = 4000.0
    G = physics.green(r * n, k) * r / np.exp(1j * k * r)
    assert np.abs(G - k * k * (np.eye(3) - np.outer(n, n))).max() < 1e-3


# --------------------------------------------------------------------------- dense system / FFT product

def test_dense_matrix_by_pairwise_loop():
    """Dense matrix entries against an explicit loop over voxel pairs (Sec. 2.1-2.2)."""
    s = w.random_mask(3, 2, 2, 0.9, 5, k=1.4, d=0.35, eps_mean=2.0 + 0.05j, eps_jitter=0.1)
    S = 0.25
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, S)
    occ = np.flatnonzero(s.mask.ravel())
    n = len(occ)
    r = system.centres(s.shape, s.d).reshape(-1, 3)
    for ii, i in enumerate(occ):
        for jj, j in enumerate(occ):
            for a in range(3):
                for b in range(3):
                    if i == j:
                        ref = physics.alpha_inv(s.eps.ravel()[i], s.k * s.d, S) if a == b else 0.0
                    else:
                        ref = -s.d ** 3 * physics.green(r[i] - r[j], s.k)[a, b]
                    assert abs(A[a * n + ii, b * n + jj] - ref) < 1e-14 * max(1.0, abs(ref))


def test_matrix_complex_symmetric_not_hermitian():
    s = w.random_mask(4, 3, 3, 0.7, 6, k=1.2, d=0.3)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, 0.1)
    assert np.abs(A - A.T).max() < 1e-15
    assert np.abs(A - A.conj().T).max() > 1e-3


@pytest.mark.parametrize("shape,seed", [((5, 6, 7), 1), ((2, 9, 4), 2), ((1, 1, 6), 3)])
def test_fft_matvec_equals_dense(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.7, seed, k=1.3, d=0.3, eps_jitter=0.05)
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(3,) + s.shape) + 1j * rng.normal(size=(3,) + s.shape)
    y1 = system.box_operator_dense(s.mask, s.eps, s.k, s.d, 0.2, x * s.mask)
    y2 = fftmatvec.fft_matvec(x * s.mask, s.mask, s.eps, s.k, s.d, 0.2)
    assert np.abs(y1 - y2).max() < 1e-12 * np.abs(y1).max()


def test_operator_rows_equal_dense():
    s = w.random_mask(6, 5, 4, 0.6, 9, k=1.0, d=0.4)
    rng = np.random.default_rng(9)
    x = (rng.normal(size=(3,) + s.shape) + 1j * rng.normal(size=(3,) + s.shape)) * s.mask
    y = system.box_operator_dense(s.mask, s.eps, s.k, s.d, 0.0, x)
    occ = np.flatnonzero(s.mask.ravel())[:5]
    rr = rows.operator_rows(occ, x, s.mask, s.eps, s.k, s.d, 0.0)
    for t, i in enumerate(occ):
        ref = np.array([y[a].ravel()[i] for a in range(3)])
        assert np.abs(rr[t] - ref).max() < 1e-12 * np.abs(ref).max()


# --------------------------------------------------------------------------- circulant preconditioner

def test_chan_formula_is_frobenius_optimal():
    """eq. Chan equals the least-squares circulant fit of the Toeplitz matrix (the
    property that defines it), and the residual is orthogonal to every circulant."""
    rng = np.random.default_rng(3)
    for l in (1, 2, 5, 8):
        t = rng.normal(size=2 * l - 1) + 1j * rng.normal(size=2 * l - 1)
        T = circulant.toeplitz_from_signed(t)
        c = circulant.chan_column(t)
        basis = np.stack([circulant.circulant_from_column(np.eye(l)[p]).ravel() for p in range(l)], axis=1)
        cls, *_ = np.linalg.lstsq(basis.astype(complex), T.ravel(), rcond=None)
        assert np.abs(c - cls).max() < 1e-12
        resid = T - circulant.circulant_from_column(c)
        assert np.abs(basis.T @ resid.ravel()).max() < 1e-12
        assert np.abs(circulant.average_wrapped(T, 0, 1) - circulant.circulant_from_column(c)).max() < 1e-13


@pytest.mark.parametrize("shape", [(4, 5, 6), (3, 4, 4), (5, 3, 2)])
def test_two_level_brute_force_equals_formula(shape):
    """Brute-force wrapped-diagonal averaging (x then y) of the full-box BTTB matrix
    equals the per-mode blocks built from eq. Chan on signed offsets (Sec. 3)."""
    k, d = 1.3, 0.3
    ati = complex(physics.alpha_inv(1.7161, k * d, 0.0))
    P = circulant.two_level_dense(shape, k, d, ati)
    B = circulant.two_level_blocks(shape, k, d, ati)
    assert np.abs(P - P.T).max() < 1e-14  # complex symmetric
    rng = np.random.default_rng(4)
    v = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    ones = np.ones(shape, dtype=np.uint8)
    z1 = circulant.apply_dense(v, ones, P)
    z2 = circulant.apply_blocks(v, ones, circulant.invert_blocks(B))
    assert np.abs(z1 - z2).max() < 1e-12 * np.abs(z1).max()


@pytest.mark.parametrize("shape", [(3, 2, 5), (2, 3, 4), (1, 2, 6), (3, 2, 1)])
def test_one_level_brute_force_equals_formula(shape):
    """The 1-level preconditioner C_B of Sec. 3: wrapped-diagonal averaging of the x-level
    Toeplitz blocks of the full-box matrix equals the per-mode dense blocks from eq. Chan
    along x and a DFT over x; it is complex symmetric, and for nx = 1 it is the matrix
    itself (nothing to average)."""
    k, d = 1.3, 0.3
    ati = complex(physics.alpha_inv(1.7161, k * d, 0.0))
    P = circulant.one_level_dense(shape, k, d, ati)
    assert np.abs(P - P.T).max() < 1e-14
    D = circulant.one_level_blocks(shape, k, d, ati)
    rng = np.random.default_rng(6)
    v = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    ones = np.ones(shape, dtype=np.uint8)
    Dinv = np.linalg.inv(D)
    z1 = circulant.apply_dense(v, ones, P)
    z2 = circulant.apply_one_level(v, ones, Dinv)
    assert np.abs(z1 - z2).max() < 1e-12 * np.abs(z1).max()
    if shape[2] == 1:
        A = system.dense_matrix(ones, np.full(shape, 1.7161, dtype=complex), k, d, 0.0)
        assert np.abs(P - A).max() < 1e-12 * np.abs(A).max()


def test_occupied_layers_preconditioner_is_the_smallest_box_one():
    """The dense level spans the occupied z layers: for a body with air layers above and
    below, M P^{-1} M equals the brute-force P of the smallest box around it (the paper's
    grid), embedded with zeros; on a box the body fills, it is the plain full-box P."""
    k, d = 1.3, 0.3
    ati = complex(physics.alpha_inv(1.7161, k * d, 0.0))
    rng = np.random.default_rng(11)
    mask = np.zeros((7, 4, 5), dtype=np.uint8)
    mask[2:5] = rng.random((3, 4, 5)) < 0.8
    mask[2, 0, 0] = mask[4, 3, 4] = 1
    assert circulant.occupied_layers(mask) == (2, 5)
    v = rng.normal(size=(3, 7, 4, 5)) + 1j * rng.normal(size=(3, 7, 4, 5))
    z0, Binv = circulant.blocks_for_mask(mask, k, d, ati)
    z = circulant.apply_blocks_layers(v, mask, Binv, z0)
    P = circulant.two_level_dense((3, 4, 5), k, d, ati)
    ref = np.zeros_like(z)
    ref[:, 2:5] = circulant.apply_dense(v[:, 2:5], mask[2:5], P)
    assert np.abs(z - ref).max() < 1e-12 * np.abs(ref).max()
    full = np.ones((3, 4, 5), dtype=np.uint8)
    z0, Binv = circulant.blocks_for_mask(full, k, d, ati)
    assert z0 == 0
    assert np.abs(circulant.apply_blocks_layers(v[:, :3], full, Binv, 0)
                  - circulant.apply_dense(v[:, :3], full, P)).max() < 1e-12 * np.abs(v).max()
    plate = w.plate_case(0.1, 1.6, 40)["scatterer"]  # fitted nz = 11, box grown to 12
    assert circulant.occupied_layers(plate.mask) == (0, plate.meta["fit_shape"][0]) == (0, 11)


def test_two_level_block_symmetries():
    """B(-wx, wy) = Sx B Sx (and likewise for y), B(w)^T = B(-w), and B commutes
    with the z-reflection R = J_n (x) diag(1, 1, -1)."""
    nz, ny, nx = 5, 6, 4
    k, d = 1.7, 0.25
    B = circulant.two_level_blocks((nz, ny, nx), k, d, 20.0 - 0.1j)
    sx = np.repeat([-1.0, 1.0, 1.0], nz)
    sy = np.repeat([1.0, -1.0, 1.0], nz)
    J = np.eye(nz)[::-1]
    Rm = np.kron(np.diag([1.0, 1.0, -1.0]), J)
    for iy in range(ny):
        for ix in range(nx):
            b = B[iy, ix]
            bx = B[iy, (-ix) % nx]
            by = B[(-iy) % ny, ix]
            bxy = B[(-iy) % ny, (-ix) % nx]
            assert np.abs(bx - sx[:, None] * b * sx[None, :]).max() < 1e-12
            assert np.abs(by - sy[:, None] * b * sy[None, :]).max() < 1e-12
            assert np.abs(b.T - bxy).max() < 1e-12
            assert np.abs(Rm @ b - b @ Rm).max() < 1e-12


def test_folded_halves_symmetric_for_even_nz():
    """With v split into even / odd parts under the z reflection, each mode block restricted
    to one half (planes iz < nz/2 with the mirror plane folded in with sign sigma s_b, plus
    the middle plane for odd nz where sigma s_b = +1) satisfies (S B_sigma)^T = S B_sigma
    with S = diag(1, 1, -1) per component when nz is even.  This is what allows storing half
    of each inverse; with odd nz the middle plane enters without the fold's factor of two and
    the symmetry is lost."""
    for (nz, ny, nx), even in (((6, 4, 5), True), ((7, 3, 4), False)):
        k, d = 1.3, 0.3
        B = circulant.two_level_blocks((nz, ny, nx), k, d, 21.0 - 0.02j)
        h = nz // 2
        s = np.array([1.0, 1.0, -1.0])
        worst = 0.0
        for iy in range(ny):
            for ix in range(nx):
                b = B[iy, ix]
                for sig in (1.0, -1.0):
                    idx = [(a, iz) for a in range(3) for iz in range(h)]
                    if nz % 2:
                        idx += [(a, h) for a in range(3) if sig * s[a] > 0]
                    half = np.empty((len(idx), len(idx)), dtype=complex)
                    for p_, (a, iz) in enumerate(idx):
                        for q_, (bb, jz) in enumerate(idx):
                            v = b[a * nz + iz, bb * nz + jz]
                            if jz < h:
                                v += sig * s[bb] * b[a * nz + iz, bb * nz + nz - 1 - jz]
                            half[p_, q_] = v
                    M = np.array([s[a] for a, _ in idx])[:, None] * half
                    worst = max(worst, np.abs(M - M.T).max() / np.abs(M).max())
        assert (worst < 1e-13) if even else (worst > 1e-3), (nz, worst)


def test_two_level_exact_for_single_column():
    """l = m = 1: both circulant levels are 1 x 1, so for a fully occupied homogeneous
    column P equals the system matrix and preconditioned GMRES converges in one step."""
    nz = 9
    s = w.cuboid_grid(1, 1, nz, k=2.0, d=0.3, m_index=1.31)
    ati = complex(physics.alpha_inv(1.31 ** 2, s.k * s.d, 0.0))
    P = circulant.two_level_dense(s.shape, s.k, s.d, ati)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, 0.0)
    assert np.abs(P - A).max() < 1e-13 * np.abs(A).max()
    Bi = circulant.invert_blocks(circulant.two_level_blocks(s.shape, s.k, s.d, ati))
    b = system.incident_field(s.mask, s.k, s.d, (0, 0, 1), (1, 0, 0))
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, 0.0)
    _, info = gmres.gmres(mv, b, precond=lambda v: circulant.apply_blocks(v, s.mask, Bi), tol=1e-12)
    assert info["iters"] == 1 and info["converged"]


def test_preconditioner_storage_count():
    """Naive 2-level storage is l m (3n)^2 entries (Sec. 3.2 costings, O(x^4))."""
    shape = (4, 5, 6)
    B = circulant.two_level_blocks(shape, 1.0, 0.3, 20.0)
    assert B.size == 6 * 5 * (3 * 4) ** 2


def test_precond_rows_equal_blocks():
    shape = (6, 5, 4)
    k, d, ati = 1.2, 0.3, 21.0 - 0.02j
    B = circulant.two_level_blocks(shape, k, d, ati)
    rng = np.random.default_rng(7)
    z = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    Vf = np.fft.fft2(z, axes=(2, 3))
    Vm = np.moveaxis(Vf, (2, 3), (0, 1)).reshape(shape[1], shape[2], 3 * shape[0])
    Pz = np.fft.ifft2(np.moveaxis(np.einsum("yxij,yxj->yxi", B, Vm).reshape(shape[1], shape[2], 3, shape[0]),
                                  (0, 1), (2, 3)), axes=(2, 3))
    idx = [0, 17, 63, 119]
    rr = rows.precond_rows(idx, z, k, d, ati)
    for t, i in enumerate(idx):
        ref = np.array([Pz[a].ravel()[i] for a in range(3)])
        assert np.abs(rr[t] - ref).max() < 1e-12 * np.abs(ref).max()


# --------------------------------------------------------------------------- GMRES

def _small_problem(g=6, x=2.0):
    s = w.hex_prism_grid(x, 1.0, g, 1.31)
    dirs, pols = w.plane_wave_z(("x",))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    return s, dirs[0], pols[0], b


def test_gmres_matches_lu_and_estimate_is_true_residual():
    s, dv, pv, b = _small_problem(8)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, 0.0)
    c = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, 0.0)
    xg, info = gmres.gmres(mv, b, restart=5, tol=1e-11)
    assert info["converged"] and info["cycles"] > 1
    assert np.abs(xg - c).max() < 1e-9 * np.abs(c).max()
    hist = np.array(info["history"])
    # within a cycle the estimate never increases
    for cyc in range(info["cycles"]):
        seg = hist[cyc * 5:(cyc + 1) * 5]
        assert np.all(np.diff(seg) <= 1e-15)
    assert abs(hist[-1] - info["rel_residual"]) < 1e-9


def test_gmres_exact_when_restart_exceeds_dimension():
    rng = np.random.default_rng(8)
    n = 12
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 5 * np.eye(n)
    b = rng.normal(size=n) + 0j
    x, info = gmres.gmres(lambda v: A @ v, b, restart=20, tol=1e-14, maxit=n)
    assert info["iters"] <= n
    assert np.abs(A @ x - b).max() < 1e-11


def test_alpha_tilde_variants_closed_forms():
    """The three readings of the preconditioner's constant diagonal (Sec. 1, Sec. 3.1) on a
    two-material body: fraction f of the voxels at eps1, the rest at eps2.  mean_eps is
    alpha^{-1}(f eps1 + (1-f) eps2); mean_alpha is f alpha^{-1}(eps1) + (1-f) alpha^{-1}(eps2);
    mode is the majority's alpha^{-1}; for a homogeneous body all three are its value."""
    rng = np.random.default_rng(5)
    kd, S = 0.4, 0.3
    mask = rng.random((6, 7, 8)) < 0.8
    e1, e2 = 1.7161 + 0.0j, 3.1684 + 0.02j
    eps = np.where(rng.random(mask.shape) < 0.7, e1, e2).astype(np.complex128)
    occ = mask.astype(bool)
    f = float(np.mean(eps[occ] == e1))
    assert 0.5 < f < 0.9
    a1 = complex(physics.alpha_inv(e1, kd, S))
    a2 = complex(physics.alpha_inv(e2, kd, S))
    am = physics.alpha_tilde_inv(eps, mask, kd, S, "mean_eps")
    assert abs(am - complex(physics.alpha_inv(f * e1 + (1 - f) * e2, kd, S))) < 1e-12 * abs(am)
    aa = physics.alpha_tilde_inv(eps, mask, kd, S, "mean_alpha")
    assert abs(aa - (f * a1 + (1 - f) * a2)) < 1e-12 * abs(aa)
    assert physics.alpha_tilde_inv(eps, mask, kd, S, "mode") == a1
    assert abs(am - aa) > 1e-3 * abs(aa)  # the readings differ for an inhomogeneous body
    hom = np.full(mask.shape, e2)
    for v in ("mean_eps", "mean_alpha", "mode"):
        assert abs(physics.alpha_tilde_inv(hom, mask, kd, S, v) - a2) < 1e-12 * abs(a2)
    # a tie goes to the smallest value, whatever the voxel order
    tie = np.ones((1, 1, 4), dtype=bool)
    for te in (np.array([[[e2, e1, e1, e2]]]), np.array([[[e1, e2, e2, e1]]])):
        assert physics.alpha_tilde_inv(te, tie, kd, S, "mode") == a1


def test_circulant_plus_diagonal_neumann_steps():
    """P = D + C (Sec. 1 P = D~ + C with the true diagonal; Sec. 5 circulant-plus-diagonal)
    applied by z = Q(v - Delta z), Q = M B^{-1} M the circulant preconditioner as applied:
    zero steps give Q itself; on a two-material body where Q Delta is a contraction the
    steps converge to the dense solve (Q^{-1} + Delta)^{-1} v on the occupied voxels, the
    error shrinking every step; for a homogeneous body Delta = 0."""
    rng = np.random.default_rng(21)
    shape = (4, 3, 5)
    k, d = 1.1, 0.3
    mask = (rng.random(shape) < 0.8).astype(np.uint8)
    e1, e2 = 1.7161 + 0.0j, 1.9 + 0.01j
    eps = np.where(rng.random(shape) < 0.6, e1, e2)
    ati = physics.alpha_tilde_inv(eps, mask, k * d, 0.0, "mean_eps")
    P = circulant.two_level_dense(shape, k, d, ati)  # alpha~^{-1} I - C2 on the whole box
    delta = circulant.diag_correction(eps, mask, k * d, 0.0, ati)
    occ = mask.astype(bool).ravel()
    sel = np.repeat(occ[None], 3, axis=0).ravel()  # box order [3][nz][ny][nx]
    Q = np.linalg.inv(P)[np.ix_(sel, sel)]  # M B^{-1} M on the occupied voxels
    Dl = np.repeat(delta.ravel()[None], 3, axis=0).ravel()[sel]
    apply_B = lambda v: circulant.apply_dense(v, mask, P)
    v = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    v = v * mask[None]
    z0 = circulant.apply_plus_diagonal(v, apply_B, delta, 0)
    assert np.allclose(z0, apply_B(v), rtol=0, atol=1e-13)
    exact = np.zeros(v.shape, dtype=np.complex128).ravel()
    exact[sel] = np.linalg.solve(np.eye(sel.sum()) + Q * Dl[None, :], Q @ v.ravel()[sel])
    exact = exact.reshape(v.shape)
    rho = max(abs(np.linalg.eigvals(Q * Dl[None, :])))
    assert rho < 0.6
    errs = [np.abs(circulant.apply_plus_diagonal(v, apply_B, delta, s) - exact).max()
            for s in (0, 4, 12, 48)]
    assert errs[-1] < 1e-8 * np.abs(exact).max()
    assert all(e2_ < e1_ for e1_, e2_ in zip(errs, errs[1:]))
    hom = np.full(shape, e1)
    dh = circulant.diag_correction(hom, mask, k * d, 0.0, complex(physics.alpha_inv(e1, k * d, 0.0)))
    assert np.abs(dh).max() < 1e-12


def _rho_q_delta(shape, e_host, e_inc, frac, seed=3, kd=0.31):
    """Spectral radius of Q Delta for a full box with a fraction `frac` of random voxels at
    e_inc in a host e_host, alpha~ from the mean permittivity."""
    rng = np.random.default_rng(seed)
    mask = np.ones(shape, np.uint8)
    eps = np.where(rng.random(shape) < frac, e_inc, e_host).astype(np.complex128)
    ati = physics.alpha_tilde_inv(eps, mask, kd, 0.0, "mean_eps")
    Q = np.linalg.inv(circulant.two_level_dense(shape, 1.0, kd, ati))
    delta = circulant.diag_correction(eps, mask, kd, 0.0, ati)
    Dl = np.repeat(delta.ravel()[None], 3, axis=0).ravel()
    return max(abs(np.linalg.eigvals(Q * Dl[None, :])))


def test_circulant_plus_diagonal_contraction_shrinks_with_box():
    """The fixed-point form of P = D + C converges only while rho(Q Delta) < 1.  For ice with
    30 % random voxels at m = 1.78 the radius grows with the box (6^3 -> 8^3), while a
    small permittivity contrast keeps it near zero: the series suits mild inhomogeneity."""
    r6 = _rho_q_delta((6, 6, 6), 1.31 ** 2, 1.78 ** 2, 0.3)
    r8 = _rho_q_delta((8, 8, 8), 1.31 ** 2, 1.78 ** 2, 0.3)
    assert 0.5 < r6 < r8 < 1.0
    assert _rho_q_delta((6, 6, 6), 1.7161, 1.75, 0.5) < 0.05


def test_left_gmres_exact_preconditioner_one_step():
    """Left preconditioning (Sec. 1, eq. general_prec) with P^{-1} = A^{-1}: P^{-1} A = I, so
    the first Krylov step solves the system; right-preconditioned GMRES does the same."""
    rng = np.random.default_rng(11)
    n = 15
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 4 * np.eye(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    Ainv = np.linalg.inv(A)
    for side in ("left", "right"):
        x, info = gmres.gmres(lambda v: A @ v, b, precond=lambda v: Ainv @ v, tol=1e-12,
                              side=side)
        assert info["converged"] and info["iters"] == 1, (side, info["iters"])
        assert np.abs(A @ x - b).max() < 1e-10 * np.abs(b).max()


def test_left_gmres_residuals_are_those_of_the_preconditioned_system():
    """Left GMRES on a small DDA system with a non-trivial P (the 2-level circulant one):
    the solution is the LU one, the reported residual is ||P^{-1}(b - A x)|| / ||P^{-1} b||
    recomputed from x, the true residual is reported beside it, and P = I reproduces
    right-preconditioned GMRES iteration for iteration."""
    s, dv, pv, b = _small_problem(8)
    S = physics.lattice_S(dv, pv)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, S)
    c = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S)
    ati = complex(physics.alpha_inv(s.eps[s.mask.astype(bool)].mean(), s.k * s.d, 0.0))
    z0, Bi = circulant.blocks_for_mask(s.mask, s.k, s.d, ati)
    pc = lambda v: circulant.apply_blocks_layers(v, s.mask, Bi, z0)
    x, info = gmres.gmres(mv, b, precond=pc, restart=8, tol=1e-11, side="left")
    assert info["converged"]
    assert np.abs(x - c).max() < 1e-8 * np.abs(c).max()
    prel = np.linalg.norm(pc(b - mv(x))) / np.linalg.norm(pc(b))
    assert abs(prel - info["rel_residual"]) < 1e-12 and prel <= 1e-11
    true = np.linalg.norm(b - mv(x)) / np.linalg.norm(b)
    assert abs(true - info["true_rel_residual"]) < 1e-13
    ident = lambda v: v
    _, il = gmres.gmres(mv, b, precond=ident, restart=6, tol=1e-6, side="left")
    _, ir = gmres.gmres(mv, b, precond=ident, restart=6, tol=1e-6, side="right")
    assert il["iters"] == ir["iters"] and np.allclose(il["history"], ir["history"], rtol=0, atol=1e-14)


# --------------------------------------------------------------------------- cross sections

def test_optical_theorem_exact_solution():
    """C_ext = C_abs + C_sca for the exact (LU) solution, lossless and lossy ice."""
    for m_index in (1.31, 1.31 + 0.05j):
        s = w.hex_prism_grid(2.5, 1.2, 6, m_index)
        dv, pv = np.array([0.3, 0.4, 0.866]), None
        dv = dv / np.linalg.norm(dv)
        pv = np.cross(dv, [0, 0, 1.0])
        pv /= np.linalg.norm(pv)
        S = physics.lattice_S(dv, pv)
        b = system.incident_field(s.mask, s.k, s.d, dv, pv)
        A = system.dense_matrix(s.mask, s.eps, s.k, s.d, S)
        c = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
        ce, ca, cs = xsec.cross_sections(c, s.mask, s.eps, s.k, s.d, dv, pv)
        assert abs(ce - ca - cs) < 1e-12 * ce
        if m_index.imag == 0:
            assert abs(ca) < 1e-14 * ce
        else:
            assert ca > 1e-3 * ce


def test_scattering_two_routes():
    """Far-field quadrature and the Im G double sum (dense and FFT) agree."""
    s, dv, pv, b = _small_problem(6, 3.0)
    rng = np.random.default_rng(11)
    c = (rng.normal(size=(3,) + s.shape) + 1j * rng.normal(size=(3,) + s.shape)) * s.mask
    c1 = xsec.c_sca_farfield(c, s.mask, s.k, s.d, n_theta=64, n_phi=128)
    c2 = xsec.c_sca_imag_dense(c, s.mask, s.k, s.d)
    c3 = xsec.c_sca_imag_sum(c, s.mask, s.k, s.d)
    assert abs(c1 - c2) < 1e-10 * c2 and abs(c3 - c2) < 1e-12 * c2


def test_single_dipole():
    """One voxel: c = alpha E0, C_ext = 4 pi k d^3 Im alpha and, for real eps,
    C_ext = C_sca = (8 pi / 3) k^4 d^6 |alpha|^2 (point-dipole textbook result)."""
    k, d = 1.0, 0.25
    s = w.cuboid_grid(1, 1, 1, k, d, 1.31)
    b = system.incident_field(s.mask, k, d, (0, 0, 1), (1, 0, 0))
    A = system.dense_matrix(s.mask, s.eps, k, d, 0.0)
    c = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    alpha = 1.0 / physics.alpha_inv(1.31 ** 2, k * d, 0.0)
    assert abs(c[0].ravel()[0] - alpha) < 1e-15
    ce, ca, cs = xsec.cross_sections(c, s.mask, s.eps, k, d, (0, 0, 1), (1, 0, 0))
    assert abs(ce - 4 * math.pi * k * d ** 3 * alpha.imag) < 1e-14 * ce
    assert abs(cs - 8 * math.pi / 3 * k ** 4 * d ** 6 * abs(alpha) ** 2) < 1e-12 * cs
    assert abs(ce - cs) < 1e-12 * ce


def test_rayleigh_limit_small_sphere():
    """A sphere with k a << 1 scatters (8 pi / 3) k^4 a^6 |(eps - 1)/(eps + 2)|^2
    (Rayleigh); the DDA error shrinks as the sphere is refined."""
    errs = []
    for g in (8, 16):
        s = w.sphere_grid(0.05, g, 1.31)
        b = system.incident_field(s.mask, s.k, s.d, (0, 0, 1), (1, 0, 0))
        mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, 0.0)
        c, info = gmres.gmres(mv, b, tol=1e-12)
        cs = xsec.c_sca_imag_sum(c, s.mask, s.k, s.d)
        aeq = (s.n_occ * s.d ** 3 * 3 / (4 * math.pi)) ** (1 / 3)
        eps = 1.31 ** 2
        ray = 8 * math.pi / 3 * s.k ** 4 * aeq ** 6 * abs((eps - 1) / (eps + 2)) ** 2
        errs.append(abs(cs / ray - 1))
    assert errs[1] < errs[0] < 0.01


# --------------------------------------------------------------------------- adjoint

def test_adjoint_gradient_vs_finite_differences():
    s = w.random_mask(3, 3, 4, 0.8, 3, k=2.0, d=0.4, eps_mean=2.0 + 0.1j, eps_jitter=0.05)
    dv, pv = (0.0, 0.0, 1.0), (1.0, 0.0, 0.0)
    _, g = adjoint.grad_cext_dense(s.mask, s.eps, s.k, s.d, dv, pv)
    occ = np.flatnonzero(s.mask.ravel())
    h = 1e-6
    for j in occ[:5]:
        def f(de):
            e = s.eps.copy()
            e.ravel()[j] += de
            return adjoint.grad_cext_dense(s.mask, e, s.k, s.d, dv, pv)[0]
        fd = (f(h) - f(-h)) / (2 * h) + 1j * (f(1j * h) - f(-1j * h)) / (2 * h)
        assert abs(g.ravel()[j] - fd) < 1e-6 * abs(fd)
    assert np.all(g[~s.mask.astype(bool)] == 0)


# --------------------------------------------------------------------------- geometry vs the paper's tables

def test_geometry_voxel_counts_match_tables_3_4():
    """Total voxels of the fit-mode plate grids vs the paper's "#Total voxels" columns
    (Tables 3-4, two significant figures): within 5% for the closer of ceil / round."""
    rows_ = [ln.split() for ln in open(os.path.join(GOLDEN, "paper_voxel_counts.txt"))
             if ln.strip() and not ln.startswith("#")]
    assert len(rows_) == 65
    for la, mu, x, tot, _ in rows_:
        best = None
        for rnd in ("ceil", "round"):
            s = w.hex_prism_fit(float(x), float(la), float(mu), rounding=rnd) if float(x) <= 20 else None
            if s is not None:
                n = s.mask.size
            else:  # large grids: count the box without building the mask
                d = 2 * math.pi / float(x) / (10 * float(mu))
                f = math.ceil if rnd == "ceil" else (lambda v: max(1, round(v)))
                n = 1
                for e in (2.0, math.sqrt(3.0), float(la)):
                    n *= max(1, f(e / d - 1e-12))
            r = n / float(tot)
            best = r if best is None or abs(r - 1) < abs(best - 1) else best
        assert 0.95 <= best <= 1.05, (la, mu, x, tot, best)


def test_torch_complex_gradient_convention():
    """For a real loss L(z), torch stores dL/dRe z + i dL/dIm z in z.grad — the convention the
    adjoint backward returns (pinned here on L = Im(a z) + |z|^2 by hand differentiation)."""
    import torch
    a = 0.7 - 1.3j
    z = torch.tensor(0.4 + 0.9j, dtype=torch.complex128, requires_grad=True)
    L = (a * z).imag + (z.abs() ** 2)
    L.backward()
    x, y = 0.4, 0.9
    dLdx = a.imag + 2 * x   # Im(a z) = a_r y + a_i x
    dLdy = a.real + 2 * y
    assert abs(z.grad.item() - (dLdx + 1j * dLdy)) < 1e-14


def test_bicgstab_matches_lu_and_is_exact_for_scaled_identity():
    """BiCGStab (Sec. 4's second solver) against LU on a small DDA system, with and without
    the 2-level preconditioner, and its one-step exactness for A = c I."""
    from oracle import bicgstab
    s = w.hex_prism_grid(1.0, 1.0, 6, 1.31)
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, 0.0)
    b = system.incident_field(s.mask, s.k, s.d, (0, 0, 1), (1, 0, 0))
    occ = s.mask.astype(bool)
    x_lu = np.linalg.solve(A, system.box_to_compact(b, s.mask))
    mv = lambda x: fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, 0.0)
    ati = complex(physics.alpha_inv(1.31 ** 2, s.k * s.d, 0.0))
    Bi = circulant.invert_blocks(circulant.two_level_blocks(s.shape, s.k, s.d, ati))
    pc = lambda v: circulant.apply_blocks(v, s.mask, Bi)
    its = {}
    for name, P in (("plain", None), ("precond", pc)):
        x, info = bicgstab.bicgstab(mv, b, precond=P, tol=1e-12, maxit=500)
        assert info["converged"] and info["rel_residual"] <= 1e-12
        xc = system.box_to_compact(x, s.mask)
        assert np.abs(xc - x_lu).max() < 1e-9 * np.abs(x_lu).max()
        assert np.all(x[:, ~occ] == 0)
        its[name] = info["iters"]
    assert its["precond"] < its["plain"]
    c = 3.0 - 0.5j
    rhs = np.arange(12, dtype=complex).reshape(3, 2, 2) + 1j
    x, info = bicgstab.bicgstab(lambda v: c * v, rhs, tol=1e-14)
    assert info["iters"] == 1 and np.abs(x - rhs / c).max() < 1e-14
