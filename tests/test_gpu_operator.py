"""GPU parity of the FFT operator and of the 2-level preconditioner against the CPU oracle.

Sizes span several FFT tiles with ragged tails, odd radices (3, 5, 7), degenerate
dimensions (1 x 1 x n columns, a single voxel), several right-hand sides with different
LDR factors S, and the full 128^3 benchmark grid via sampled rows.
"""

import numpy as np
import pytest

import workloads as w
from gpu_helpers import make_problem, oracle_precond, rand_field, random_waves, rel_err, to_dev
from oracle import circulant, fftmatvec, physics, rows, system

pytestmark = pytest.mark.gpu

OP_CASES = [
    ((5, 6, 7), 0.7, 1),
    ((9, 4, 12), 0.6, 2),
    ((16, 16, 16), 0.65, 3),
    ((3, 10, 14), 0.8, 4),
    ((1, 1, 6), 1.0, 5),
    ((1, 1, 1), 1.0, 6),
    ((7, 5, 3), 0.5, 7),
    ((12, 20, 9), 0.7, 8),
    # z lengths 64, 128, 256 (register z pass splits 8 x 8, 8 x 16, 16 x 16), ragged tiles, a
    # 1 x 1 column
    ((32, 6, 9), 0.7, 9),
    ((64, 5, 3), 0.6, 10),
    ((128, 3, 4), 0.7, 11),
    ((32, 1, 1), 1.0, 12),
    # z lengths 36 .. 224 that are not powers of two: the mixed-radix register z pass, one
    # case per (G, P) split shape (P <= G with idle threads, P = 2 G with two frequency
    # columns per thread), ragged tiles and a 1 x 1 column
    ((18, 5, 7), 0.7, 13),
    ((20, 3, 9), 0.6, 14),
    ((24, 7, 5), 0.7, 15),
    ((40, 4, 6), 0.7, 16),
    ((48, 3, 5), 0.8, 17),
    ((56, 2, 3), 0.7, 18),
    ((72, 3, 2), 0.7, 19),
    ((80, 2, 3), 0.6, 20),
    ((96, 3, 3), 0.7, 21),
    ((98, 2, 2), 0.7, 22),
    ((112, 2, 2), 0.7, 23),
    ((48, 1, 1), 1.0, 24),
    ((36, 4, 5), 0.7, 25),
    ((256, 2, 3), 0.7, 26),
    # x and y lengths 40, 48, 56, 80, 96: the compile-time mixed-radix plans of the row and
    # strided passes (padded lengths 80, 96, 112, 160, 192; radices 3, 5, 7)
    ((3, 40, 56), 0.7, 27),
    ((2, 80, 48), 0.7, 28),
    ((2, 96, 40), 0.6, 29),
    ((2, 5, 96), 0.7, 30),
    ((3, 4, 80), 0.7, 31),
]


@pytest.mark.parametrize("shape,fill,seed", OP_CASES)
def test_operator_fp64_vs_oracle(shape, fill, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, fill, seed, k=1.3, d=0.3, eps_jitter=0.05)
    dirs, pols = random_waves(2, seed)
    with make_problem(s, max_rhs=2, precond=0) as prob:
        x = rand_field(shape, 2, seed)  # unmasked: air entries must pass through
        y = prob.apply_operator(to_dev(x), dirs, pols).cpu().numpy()
    for r in range(2):
        S = physics.lattice_S(dirs[r], pols[r])
        ref = fftmatvec.fft_matvec(x[r], s.mask, s.eps, s.k, s.d, S)
        assert rel_err(y[r], ref) < 1e-10, (shape, r)


@pytest.mark.parametrize("shape,fill,seed", [((4, 5, 6), 0.7, 11), ((6, 3, 5), 0.9, 12)])
def test_operator_vs_dense_matrix(shape, fill, seed):
    """Against the dense matrix assembled pair by pair (independent of any FFT)."""
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, fill, seed, k=2.1, d=0.25, eps_mean=3.1 + 0.2j, eps_jitter=0.1)
    dirs, pols = random_waves(1, seed)
    with make_problem(s, precond=0) as prob:
        x = rand_field(shape, 1, seed, s.mask)
        y = prob.apply_operator(to_dev(x), dirs[:1], pols[:1]).cpu().numpy()
    S = physics.lattice_S(dirs[0], pols[0])
    ref = system.box_operator_dense(s.mask, s.eps, s.k, s.d, S, x[0])
    assert rel_err(y[0], ref) < 1e-10


@pytest.mark.parametrize("shape,force", [((16, 5, 7), "1,3"), ((16, 5, 7), "8,8"),
                                         ((48, 3, 5), "4,5"), ((48, 3, 5), "1,1"),
                                         ((64, 4, 3), "2,2"), ((128, 2, 3), "4,8")])
def test_operator_register_zpass_schedules(shape, force, monkeypatch):
    """The register z pass under forced tile widths and items per workgroup: several items per
    workgroup with the next one's loads in flight, ragged last chunks, rows without a distinct
    ky mirror; 5 right-hand sides, FP64 and FP32, against the oracle."""
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.7, 71, k=1.3, d=0.3, eps_jitter=0.05)
    dirs, pols = random_waves(5, 71)
    dirs, pols = dirs[:5], pols[:5]
    x = rand_field(shape, 5, 71)
    monkeypatch.setenv("DDA_ZPASS_FORCE", force)
    with make_problem(s, precond=0, max_rhs=5) as prob:
        y64 = prob.apply_operator(to_dev(x), dirs, pols).cpu().numpy()
        y32 = prob.apply_operator(to_dev(x), dirs, pols, fp32=True).cpu().numpy()
    for r in range(5):
        S = physics.lattice_S(dirs[r], pols[r])
        ref = fftmatvec.fft_matvec(x[r], s.mask, s.eps, s.k, s.d, S)
        assert rel_err(y64[r], ref) < 1e-10, (force, r)
        assert rel_err(y32[r], ref) < 1e-5, (force, r)
    monkeypatch.setenv("DDA_ZPASS_FORCE", "3,1")  # not a power of two: rejected at create
    with pytest.raises(Exception, match="DDA_ZPASS_FORCE"):
        make_problem(s, precond=0, max_rhs=5)


@pytest.mark.parametrize("shape,seed", [((5, 6, 7), 21), ((16, 16, 16), 22), ((12, 20, 9), 23),
                                        ((64, 6, 5), 24), ((128, 4, 3), 25), ((40, 5, 6), 26),
                                        ((96, 4, 3), 27), ((72, 3, 4), 28), ((256, 3, 2), 29),
                                        ((3, 40, 56), 30), ((2, 80, 48), 31), ((2, 96, 40), 32),
                                        ((2, 5, 96), 33), ((3, 4, 80), 34)])
def test_operator_fp32_vs_oracle(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.7, seed, k=1.3, d=0.3)
    dirs, pols = random_waves(1, seed)
    with make_problem(s, precond=0, precision=1) as prob:
        x = rand_field(shape, 1, seed, s.mask)
        y = prob.apply_operator(to_dev(x), dirs[:1], pols[:1], fp32=True).cpu().numpy()
    ref = fftmatvec.fft_matvec(x[0], s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    assert rel_err(y[0], ref) < 1e-5


PC_CASES = [((4, 5, 6), 31), ((5, 4, 3), 32), ((7, 6, 10), 33), ((1, 3, 4), 34),
            ((16, 16, 16), 35), ((9, 8, 12), 36), ((3, 1, 1), 37), ((2, 7, 5), 38),
            # half-block orders above 256: the 512-thread Gauss-Jordan kernel, even and odd nz
            ((200, 2, 3), 39), ((175, 2, 2), 40),
            # unpadded x and y lengths 40 .. 96 of the preconditioner's compile-time plans
            ((4, 6, 80), 41), ((3, 96, 5), 42), ((2, 40, 56), 43), ((3, 48, 96), 44)]


@pytest.mark.parametrize("shape,seed", PC_CASES)
def test_preconditioner_fp64_vs_oracle(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.75, seed, k=1.1, d=0.35, eps_jitter=0.05)
    with make_problem(s, precond=2, max_rhs=3) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 3, seed)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    pc = oracle_precond(s)
    for r in range(3):
        ref = pc(x[r])
        assert rel_err(z[r], ref) < 1e-10, (shape, r)


@pytest.mark.parametrize("fp32,nrhs,shape,seed", [(0, 6, (6, 8, 10), 81), (1, 6, (6, 8, 10), 82),
                                                  (1, 9, (8, 6, 5), 83), (0, 5, (16, 12, 10), 84)])
def test_preconditioner_many_rhs_vs_oracle(fp32, nrhs, shape, seed):
    """More right-hand sides than one column block: the block product streams each tile for
    2 (FP64) or 4 (FP32) blocks of 8 columns, over several chunks with a ragged last one."""
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.75, seed, k=1.2, d=0.3, eps_jitter=0.05)
    with make_problem(s, precond=2, max_rhs=nrhs, precision=fp32) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, nrhs, seed)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    pc = oracle_precond(s)
    for r in range(nrhs):
        assert rel_err(z[r], pc(x[r])) < (1e-5 if fp32 else 1e-10), (shape, r)


@pytest.mark.parametrize("shape,z0,z1,seed", [((10, 8, 12), 2, 7, 61), ((9, 6, 10), 1, 7, 62),
                                               ((12, 16, 16), 3, 11, 63), ((7, 5, 6), 0, 5, 64)])
def test_preconditioner_spans_occupied_layers(shape, z0, z1, seed):
    """A box with air layers above and below the body: the dense level spans the occupied
    layers only (even and odd extents), as for the paper's smallest box around the body."""
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.7, seed, k=1.3, d=0.3, eps_jitter=0.05)
    air = np.ones(nz, dtype=bool)
    air[z0:z1] = False
    s.mask[air] = 0
    s.eps[air] = 1.0
    assert s.mask[z0].any() and s.mask[z1 - 1].any()
    assert circulant.occupied_layers(s.mask) == (z0, z1)
    with make_problem(s, precond=2, max_rhs=2) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 2, seed)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    pc = oracle_precond(s)
    for r in range(2):
        assert rel_err(z[r], pc(x[r])) < 1e-10, (shape, r)
        assert np.all(z[r][:, air] == 0)


ONE_LEVEL_CASES = [((4, 5, 12), 0, 1, 91), ((3, 2, 16), 0, 3, 92), ((6, 4, 9), 1, 1, 93),
                   ((2, 3, 7), 0, 2, 94), ((1, 1, 8), 0, 1, 95), ((16, 16, 6), 0, 2, 96),
                   ((5, 6, 10), 1, 3, 97)]


@pytest.mark.parametrize("shape,fp32,nrhs,seed", ONE_LEVEL_CASES)
def test_one_level_preconditioner_vs_oracle(shape, fp32, nrhs, seed):
    """The 1-level preconditioner (precond = 1, Sec. 3 C_B): x-mode blocks of order 3 nz ny,
    odd and even nx, one and several right-hand sides, FP64 and FP32."""
    from oracle import circulant
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.75, seed, k=1.2, d=0.3, eps_jitter=0.05)
    with make_problem(s, precond=1, max_rhs=nrhs, precision=fp32) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, nrhs, seed)
        z = prob.apply_preconditioner(to_dev(x), fp32=bool(fp32)).cpu().numpy()
    occ = s.mask.astype(bool)
    ati = complex(physics.alpha_inv(s.eps[occ].mean(), s.k * s.d, 0.0))
    Dinv = np.linalg.inv(circulant.one_level_blocks(shape, s.k, s.d, ati))
    for r in range(nrhs):
        ref = circulant.apply_one_level(x[r], s.mask, Dinv)
        assert rel_err(z[r], ref) < (1e-5 if fp32 else 1e-10), (shape, r)


def test_one_level_solve_and_limits():
    """GMRES with the 1-level preconditioner reaches the dense-LU solution on a cuboid
    elongated along x, and blocks above order 768 are refused."""
    from paper_1903_09802_amd.dda import DDAError
    from oracle import system
    s = w.cuboid_grid(24, 4, 4, 1.5, 0.25, 1.31)
    dirs, pols = random_waves(1, 98)
    dirs, pols = dirs[:1], pols[:1]
    A = system.dense_matrix(s.mask, s.eps, s.k, s.d, physics.lattice_S(dirs[0], pols[0]))
    b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])
    cref = system.compact_to_box(np.linalg.solve(A, system.box_to_compact(b, s.mask)), s.mask)
    its = {}
    for precond in (0, 1, 2):
        with make_problem(s, precond=precond, tol=1e-11) as prob:
            if precond:
                prob.build_preconditioner(0.0)
            out = prob.solve(dirs, pols)
        assert out["stats"][0]["converged"] == 1
        assert rel_err(out["c"][0].cpu().numpy(), cref) < 1e-9, precond
        its[precond] = out["stats"][0]["iters"]
    assert its[1] < its[0], its
    s = w.cuboid_grid(4, 16, 18, 1.0, 0.3, 1.31)  # 3 nz ny = 864
    with make_problem(s, precond=1) as prob:
        with pytest.raises(DDAError) as ei:
            prob.build_preconditioner(0.0)
        assert ei.value.status == -5


def test_preconditioner_brute_force_definition():
    """Against P built by wrapped-diagonal averaging of the full-box BTTB matrix."""
    shape = (4, 5, 6)
    s = w.random_mask(6, 5, 4, 0.8, 41, k=1.6, d=0.3)
    assert circulant.occupied_layers(s.mask) == (0, 4)  # the dense level spans the box
    occ = s.mask.astype(bool)
    ati = complex(physics.alpha_inv(s.eps[occ].mean(), s.k * s.d, 0.25))
    P = circulant.two_level_dense(shape, s.k, s.d, ati)
    with make_problem(s, precond=2) as prob:
        prob.build_preconditioner(0.25)
        x = rand_field(shape, 1, 41)
        z = prob.apply_preconditioner(to_dev(x)).cpu().numpy()
    ref = circulant.apply_dense(x[0], s.mask, P)
    assert rel_err(z[0], ref) < 1e-10


@pytest.mark.parametrize("shape,seed", [((5, 6, 7), 51), ((16, 16, 16), 52), ((200, 3, 2), 53),
                                        ((175, 2, 2), 54)])
def test_preconditioner_fp32_vs_oracle(shape, seed):
    nz, ny, nx = shape
    s = w.random_mask(nx, ny, nz, 0.7, seed, k=1.3, d=0.3)
    with make_problem(s, precond=2, precision=1) as prob:
        prob.build_preconditioner(0.0)
        x = rand_field(shape, 1, seed)
        z = prob.apply_preconditioner(to_dev(x), fp32=True).cpu().numpy()
    ref = oracle_precond(s)(x[0])
    assert rel_err(z[0], ref) < 1e-5


def test_operator_full_size_sampled_rows():
    """128^3 benchmark prism (padded 256^3), FP64: sampled rows by direct summation."""
    cfg = w.config_c2()
    s = cfg["scatterer"]
    dirs, pols = cfg["dirs"], cfg["pols"]
    with make_problem(s, precond=0, max_rhs=2) as prob:
        x = rand_field(s.shape, 2, 61, s.mask)
        y = prob.apply_operator(to_dev(x), dirs, pols).cpu().numpy()
    occ = np.flatnonzero(s.mask.ravel())
    rng = np.random.default_rng(61)
    samples = np.concatenate([occ[[0, len(occ) // 2, -1]], rng.choice(occ, 3, replace=False)])
    for r in range(2):
        S = physics.lattice_S(dirs[r], pols[r])
        ref = rows.operator_rows(samples, x[r], s.mask, s.eps, s.k, s.d, S)
        got = np.stack([[y[r][a].ravel()[i] for a in range(3)] for i in samples])
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), r


def test_operator_96_prism_sampled_rows():
    """The largest prism grid of the batch workload, 96^3 (z length 192 = 16 x 12, the
    mixed-radix register z pass), FP64 and FP32: sampled rows by direct summation."""
    s = w.hex_prism_grid(19.0, 1.0, 96, 1.31)
    dirs, pols = random_waves(2, 63)
    occ = np.flatnonzero(s.mask.ravel())
    rng = np.random.default_rng(63)
    samples = np.concatenate([occ[[0, len(occ) // 2, -1]], rng.choice(occ, 3, replace=False)])
    x = rand_field(s.shape, 2, 63, s.mask)
    with make_problem(s, precond=0, max_rhs=2) as prob:
        for fp32, tol in ((0, 1e-10), (1, 2e-5)):
            y = prob.apply_operator(to_dev(x), dirs, pols, fp32=fp32).cpu().numpy()
            for r in range(2):
                S = physics.lattice_S(dirs[r], pols[r])
                ref = rows.operator_rows(samples, x[r], s.mask, s.eps, s.k, s.d, S)
                got = np.stack([[y[r][a].ravel()[i] for a in range(3)] for i in samples])
                assert np.abs(got - ref).max() < tol * np.abs(ref).max(), (fp32, r)


def test_preconditioner_full_size_sampled_rows():
    """128^3 homogeneous cuboid: z = P^{-1} v, checked by evaluating sampled rows of P z."""
    n = 128
    k, d = 20.0, 2.0 / n
    s = w.cuboid_grid(n, n, n, k, d, 1.31)
    ati = complex(physics.alpha_inv(1.31 ** 2, k * d, 0.0))
    with make_problem(s, precond=2) as prob:
        prob.build_preconditioner(0.0)
        v = rand_field(s.shape, 1, 62)
        z = prob.apply_preconditioner(to_dev(v)).cpu().numpy()
    rng = np.random.default_rng(62)
    samples = np.concatenate([[0, n ** 3 - 1], rng.choice(n ** 3, 3, replace=False)])
    gen = circulant.two_level_generator(s.shape, k, d)
    Pz = rows.precond_rows(samples, z[0], k, d, ati, generator=gen)
    ref = np.stack([[v[0][a].ravel()[i] for a in range(3)] for i in samples])
    assert np.abs(Pz - ref).max() < 1e-9 * np.abs(ref).max()
