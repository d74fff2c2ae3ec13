/*
 * dda.h — C-ABI of the MI355X (gfx950) preconditioned discrete dipole approximation solver.
 *
 * Method: Groth, Polimeridis & White, "Preconditioning the discrete dipole
 * approximation".  A voxelised non-magnetic dielectric body with per-voxel
 * relative permittivity eps is illuminated by a plane wave; the unknown
 * polarisation coefficients c (Sec. 2.1, the pulse-basis expansion and the
 * collocation system) solve
 *
 *     [diag(alpha^{-1}) - d^3 G] c = E^inc                (Sec. 2.2, 3x3 block system)
 *
 * where alpha is the LDR polarisability with the voxel volume omitted
 * (Sec. 2.1), G the dyadic Green tensor between voxel centres (Sec. 2,
 * midpoint rule eq. midpoint) and E^inc = pol * exp(i k dir . r).  The
 * off-diagonal part is applied by a zero-padded 3-D FFT convolution (the
 * BTTB structure, Sec. 1 and 2.2); the system is solved by restarted GMRES,
 * optionally right-preconditioned by the 2-level circulant approximation
 * C_B2 = alpha~^{-1} I - d^3 C~_B2 (Sec. 3, eq. Chan applied along x and y,
 * dense 3n x 3n blocks along z, Sec. 3.1).
 *
 * Conventions (all functions):
 *  - Grid nx x ny x nz, arrays C-ordered [nz][ny][nx] (x fastest).  Voxel
 *    (ix,iy,iz) has centre ((ix-(nx-1)/2) d, (iy-(ny-1)/2) d, (iz-(nz-1)/2) d).
 *  - complex numbers are interleaved (re, im) pairs of double: a "c128" array
 *    of n entries is 2n doubles.
 *  - A field vector is c128 [3][nz][ny][nx] (component-major); a batch of
 *    nrhs vectors is c128 [nrhs][3][nz][ny][nx].  Entries at air voxels
 *    (mask == 0) carry no unknowns: outputs hold 0 there.
 *  - Pointers named *_dev are device (HIP) memory owned by the caller; *_host
 *    are host memory owned by the caller.  Nothing is retained after a call
 *    returns except inside the opaque handle.
 *  - nx, ny, nz must each factor into 2, 3, 5 and 7 (the FFT radices) and be
 *    at most 512.
 *  - Every function returns a dda_status; on a negative status a
 *    human-readable reason is available from dda_last_error() (per thread).
 *    No C++ exception crosses this boundary.
 *  - Work is enqueued on the HIP stream given to dda_create.  dda_solve,
 *    dda_grad_cext, dda_cross_sections and dda_build_preconditioner return
 *    after their work has completed (they produce host results);
 *    dda_apply_operator / dda_apply_preconditioner are stream-ordered and do
 *    not synchronise.
 *  - A handle is not thread-safe; distinct handles may be used concurrently.
 */
#ifndef DDA_H
#define DDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dda_problem dda_problem;

typedef enum {
  DDA_OK = 0,
  DDA_NOT_CONVERGED = 1,  /* warning: iteration cap reached; outputs hold the last iterate */
  DDA_EINVAL = -1,        /* bad argument (message says which) */
  DDA_ENOMEM = -2,        /* a device allocation failed or would exceed the size limits */
  DDA_EDEVICE = -3,       /* a HIP call failed, or a non-finite residual appeared */
  DDA_ESTATE = -4,        /* call made in the wrong state (e.g. no preconditioner built) */
  DDA_EUNSUPPORTED = -5   /* grid size outside what the FFT supports */
} dda_status;

typedef struct {
  int restart;      /* GMRES restart length m of GMRES(m), 1 .. 1023; default 30 */
  int max_iter;     /* cap on total GMRES iterations (inner ones in refinement mode); default 2000 */
  double tol;       /* stop when ||b - A x||_2 / ||b||_2 <= tol (true residual, FP64); default 1e-5 */
  int precond;      /* 0: none; 1: 1-level circulant preconditioner (Sec. 3, C_B: circulant along
                       x, a dense 3 nz ny block per x mode, 3 nz ny <= 768); 2: 2-level circulant
                       preconditioner (Sec. 3.1, circulant along x and y); default 2 */
  int precision;    /* 0: everything in FP64;
                       1: operator and preconditioner applied in FP32 (complex64) inside
                          FP64 iterative refinement: every restart cycle builds its Krylov
                          space with the FP32 operator and preconditioner on an FP64 basis
                          (FP64 Arnoldi), and every restart recomputes b - A x with the FP64
                          operator, so each cycle is one refinement step.  default 0 */
  int max_rhs;      /* largest nrhs accepted by dda_solve / dda_apply_*; sizes the workspace; default 1 */
  int solver;       /* 0: restarted GMRES(restart); 1: BiCGStab (Sec. 4's second solver), right-
                       preconditioned, restarted from the true residual when the updated one
                       has drifted or broken down; needs precision 0 and restart >= 7 (its eight
                       work vectors use the basis storage).  default 0 */
  int dense_axis;   /* axis (0 x, 1 y, 2 z) along which the 2-level preconditioner keeps dense
                       blocks; the other two axes are the circulant levels.  The paper makes x
                       and y circulant for plates and suggests the long axis of an elongated
                       prism as a circulant level instead (Sec. 5).  The library then works in
                       the cyclically rotated frame whose z axis is dense_axis; every buffer at
                       this interface stays in the caller's [.][3][nz][ny][nx] layout and
                       frame.  default 2 */
  int left_precond; /* GMRES only.  0: right preconditioning, A P^{-1} u = b, stopping on the
                       true residual ||b - A x|| / ||b||.  1: left preconditioning, the paper's
                       P^{-1} A x = P^{-1} b (Sec. 1, eq. general_prec): the Krylov space is
                       that of P^{-1} A and every stopping test (per iteration and at each
                       restart) is on ||P^{-1}(b - A x)|| / ||P^{-1} b||; dda_stats still
                       reports the true residual.  No effect without a preconditioner.
                       default 0 */
  int alpha_avg;    /* the constant diagonal alpha~^{-1} of the circulant preconditioners
                       (Sec. 1, Sec. 3.1), from the occupied voxels: 0: 1/alpha of the mean
                       permittivity; 1: the mean of 1/alpha (the diagonal averaged); 2: 1/alpha
                       of the most frequent permittivity (the paper's modal average, over the
                       body; a tie goes to the smallest value, real part first).  All equal the
                       body's value for a homogeneous body.  default 0 */
  int diag_steps;   /* 0 .. 32.  k > 0 makes the preconditioner the circulant-plus-diagonal
                       P = D + C: the circulant part C of the chosen preconditioner with the
                       true diagonal D = diag(1/alpha_j) of the occupied voxels (at the lattice
                       factor the preconditioner is built with) in place of alpha~^{-1} I
                       (Sec. 1, P = D~ + C; Sec. 5).  With Q the circulant preconditioner as
                       applied (occupied voxels in and out) and Delta = D - alpha~^{-1} I, a
                       preconditioner application returns z_k of z_0 = Q v,
                       z_{i+1} = Q (v - Delta z_i): k + 1 circulant applications, the Neumann
                       series of (I + Q Delta)^{-1} Q truncated after k + 1 terms.  Useful where
                       Q Delta is a contraction (moderate permittivity contrast); 0 is the
                       circulant preconditioner itself.  Needs a preconditioner (precond 1 or
                       2).  default 0 */
  int graph;        /* GMRES only.  Every step decides on the device whether each right-hand
                       side continues (its residual estimate against tol, breakdown, the step
                       cap, the end of the cycle), so a restart cycle needs the host once, at
                       its end.  1: each cycle is captured once into a HIP graph (per
                       right-hand-side count and precision) and replayed; 0: the same kernels
                       are launched one by one.  With per-kernel profiling on
                       (dda_profile_enable) cycles are always launched one by one.  default 1 */
} dda_options;

typedef struct {
  int iters;           /* solver iterations: GMRES steps (summed over refinement steps), or
                          BiCGStab iterations of two operator and two preconditioner applications */
  int cycles;          /* GMRES restart cycles, or BiCGStab runs from a true residual */
  int refinements;     /* FP64 refinement steps = restart cycles (precision 1), else 0 */
  int converged;       /* 1 if rel_residual <= tol */
  double rel_residual; /* final true residual ||b - A x|| / ||b||, FP64 */
  double t_setup;      /* seconds spent in dda_create for this handle (operator set-up) */
  double t_build;      /* seconds of the handle's last dda_build_preconditioner, 0 if none */
  double t_solve;      /* wall-clock seconds of this call */
  double *history;     /* in: NULL, or a caller-owned host array of history_cap doubles that
                          receives the residual after each iteration, relative to the norm the
                          stopping test uses (Sec. 4 plots these): the GMRES least-squares
                          estimate of ||b - A x|| / ||b|| (of ||P^{-1}(b - A x)|| / ||P^{-1} b||
                          when left preconditioned), or BiCGStab's updated residual */
  int history_cap;     /* in: capacity of history (at most 65536 GMRES steps are kept) */
  int history_len;     /* out: entries written, min(iters, history_cap) */
} dda_stats;

/* Fill *opt with the defaults listed above. */
void dda_default_options(dda_options *opt);

/*
 * The lattice factor S = sum_j (dir_j pol_j)^2 of each incident wave (Sec. 2.1, the LDR
 * polarisability's dependence on the direction and polarisation), and their mean: the s_bar to
 * build one preconditioner for a batch of waves with (its constant diagonal is the LDR value
 * at s_bar).  dir_host, pol_host: double [nrhs][3], checked as in dda_solve.  S_host: optional
 * host double [nrhs]; S_mean: optional host double.  Errors: EINVAL (nrhs < 1, bad vectors).
 */
dda_status dda_lattice_factor(int nrhs, const double *dir_host, const double *pol_host,
                              double *S_host, double *S_mean);

/* Reason for the last failure on this thread ("" if none).  Static storage. */
const char *dda_last_error(void);

/*
 * Create a problem: uploads nothing from the host; copies mask_dev (uint8
 * [nz][ny][nx], non-zero = occupied) and eps_dev (c128 [nz][ny][nx], relative
 * permittivity, read at occupied voxels only) into the handle, then assembles
 * the operator: the Green tensor d^3 G at every signed voxel offset (the
 * content of Algorithm 1, evaluated directly at signed offsets), its circulant
 * embedding on the 2nx x 2ny x 2nz grid and its FFT, kept as one octant of
 * six components (the per-level parities of Table 1 give the rest).
 *  k > 0: wavenumber; d > 0: voxel edge; opt may be NULL (defaults);
 *  stream: a hipStream_t (NULL = default stream).
 * Creation also times the fused z-FFT pass's launch shapes on this grid (once
 * per grid shape and process); the environment variable DDA_ZPASS_FORCE="tw,ipw"
 * replaces that choice by tw octant columns per tile and ipw items per
 * workgroup (for tests and benchmarks of that pass).
 * Errors: EINVAL (sizes < 1, k or d <= 0, no occupied voxel, an occupied voxel
 * with eps == 1 or eps == -2 where the polarisability is undefined, a malformed
 * or out-of-range DDA_ZPASS_FORCE); EUNSUPPORTED (a dimension not 7-smooth or
 * > 512); ENOMEM; EDEVICE.
 */
dda_status dda_create(int nx, int ny, int nz, const uint8_t *mask_dev, const double *eps_dev,
                      double k, double d, const dda_options *opt, void *stream,
                      dda_problem **out);

/*
 * Build the 2-level circulant preconditioner (Sec. 3, 3.1): eq. Chan along x
 * then y on the signed-offset kernel, FFTs along x and y, one dense 3nz x 3nz
 * block per Fourier mode with alpha~^{-1} on its diagonal, and explicit block
 * inverses: for even nz (complex symmetric half blocks) by the blocked symmetric
 * sweep with partial pivoting inside each 16 x 16 diagonal block, redone by
 * Gauss-Jordan elimination with partial pivoting if a diagonal block needs a
 * pivot from outside it; for odd nz by Gauss-Jordan.  alpha~ is the
 * LDR polarisability averaged over the occupied voxels as opt.alpha_avg says
 * (the "ice" value for a homogeneous body, Sec. 3.1) with lattice factor
 * S = s_bar.  Only the
 * (nx/2+1)(ny/2+1) modes with non-negative frequencies are inverted; the
 * block symmetries under x, y and z reflections supply the rest exactly.  The
 * dense z level spans the box's occupied z layers.
 * With opt.precond = 1 it builds instead the 1-level preconditioner C_B of Sec. 3:
 * eq. Chan along x only, an FFT along x, and one dense (3 nz ny)^2 block per x mode
 * (nx/2+1 inverted, the x reflection supplies the rest).
 * Stored in FP64 (precision 0) or FP32 (precision 1).
 * Errors: EINVAL (s_bar outside [0,1]); ENOMEM; EDEVICE (a singular block);
 * EUNSUPPORTED (1-level blocks of order 3 nz ny above 768).
 */
dda_status dda_build_preconditioner(dda_problem *p, double s_bar);

/*
 * Solve for nrhs incident plane waves at once.
 *  dir_host, pol_host: double [nrhs][3]; unit propagation directions and real
 *    unit polarisations orthogonal to them (|.| = 1 and dir.pol = 0 within 1e-9).
 *    Each wave has its own LDR factor S = sum_j (dir_j pol_j)^2 (Sec. 2.1), hence
 *    its own diagonal.
 *  x0_dev: optional initial guess c128 [nrhs][3][nz][ny][nx] (NULL = zero).
 *  c_dev: optional output polarisations c128 [nrhs][3][nz][ny][nx] (NULL = not returned).
 *  cext, cabs, csca: optional host double [nrhs] (NULL = not computed):
 *    C_ext = 4 pi k d^3 sum Im(E^inc* . c),
 *    C_abs = 4 pi k d^3 sum |c|^2 (-Im alpha^{-1} - (2/3)(k d)^3),
 *    C_sca = 4 pi k d^3 [(2/3)(k d)^3 sum |c|^2 + sum_{i!=j} c_i^H d^3 Im G(r_i - r_j) c_j]
 *    (Draine-Flatau forms for this scaling; |E_0| = 1; area in length units^2).
 *  stats: optional host dda_stats [nrhs]; history / history_cap are read, the rest written.
 * The solve allocates no device memory: every buffer it uses was allocated by dda_create or
 * dda_build_preconditioner.
 * Returns OK when every right-hand side reached tol, NOT_CONVERGED (outputs
 * valid) when some hit max_iter.  Errors: EINVAL (nrhs < 1 or
 * > max_rhs, bad vectors), ESTATE (opt.precond == 2 and no preconditioner
 * built), EDEVICE (non-finite residual, HIP failure).
 */
dda_status dda_solve(dda_problem *p, int nrhs, const double *dir_host, const double *pol_host,
                     const double *x0_dev, double *c_dev, double *cext, double *cabs,
                     double *csca, dda_stats *stats);

/*
 * y = A x for the full-box operator: on occupied voxels
 * y = alpha^{-1} x - d^3 G * (M x) (the system matrix of Sec. 2.2), and y = x
 * at air voxels.  x_dev, y_dev: c128 [nrhs][3][nz][ny][nx] (must not alias);
 * dir/pol as in dda_solve (they fix alpha^{-1} through S).  fp32 != 0 runs
 * the FFT product in FP32 with FP64 input and output.
 */
dda_status dda_apply_operator(dda_problem *p, int nrhs, const double *dir_host,
                              const double *pol_host, const double *x_dev, double *y_dev,
                              int fp32);

/*
 * y = M P^{-1} M x with P the circulant preconditioner opt.precond selects
 * (Sec. 3 1-level, Sec. 3.1 2-level) and M the occupancy mask (air entries of
 * y are 0); with opt.diag_steps = k > 0, the k-step circulant-plus-diagonal
 * approximation described at dda_options.  x_dev, y_dev: c128
 * [nrhs][3][nz][ny][nx] (may alias).  fp32 selects the FP32 blocks and must
 * match the precision the preconditioner was built in (else ESTATE).
 */
dda_status dda_apply_preconditioner(dda_problem *p, int nrhs, const double *x_dev,
                                    double *y_dev, int fp32);

/*
 * Cross sections (formulas as in dda_solve) of given polarisations c_dev
 * (c128 [nrhs][3][nz][ny][nx]) for the waves dir/pol.  Host outputs [nrhs],
 * each optional.
 */
dda_status dda_cross_sections(dda_problem *p, int nrhs, const double *dir_host,
                              const double *pol_host, const double *c_dev, double *cext,
                              double *cabs, double *csca);

/*
 * For callers that cannot allocate memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): C_ext and C_abs as dda_cross_sections computes them,
 * with no allocation of any kind, device or host, in the call.  Its only scratch (per-block
 * partial sums and the totals) lives in one static device array of 256.5 KiB per GPU, held
 * until the process ends; its address is looked up once per device by dda_create.
 *  nrhs: 1 .. min(max_rhs, 16) (the array holds 16 waves; larger nrhs is EINVAL).
 *  dir_host, pol_host: double [nrhs][3] as in dda_solve.  c_dev: c128 [nrhs][3][nz][ny][nx]
 *  (read at occupied voxels).  cext, cabs: optional host double [nrhs].
 * The handle's device must be current (EDEVICE otherwise).  Calls on one GPU share the array:
 * calls that overlap in time on one GPU (other streams, other threads) race; sequential calls
 * need nothing cleared, as every call overwrites all of the array it reads.
 * Errors: EINVAL, EDEVICE, ESTATE (array address not resolved on this device).
 */
dda_status dda_cross_sections_noalloc(dda_problem *p, int nrhs, const double *dir_host,
                                      const double *pol_host, const double *c_dev, double *cext,
                                      double *cabs);

/*
 * Gradient of C_ext with respect to the per-voxel permittivity, by one forward
 * and one adjoint solve with the same operator and preconditioner (the
 * matrix is complex symmetric, Sec. 2.2, so the adjoint system is A lambda =
 * conj(E^inc)).  grad_dev: c128 [nz][ny][nx] receiving dC/dRe(eps) +
 * i dC/dIm(eps) at occupied voxels and 0 in air.  cext: optional host double.
 * stats: optional host dda_stats [2] (forward, adjoint).  Both solves use the handle's
 * buffers (the forward solution is kept in one allocated by dda_create): no allocation.
 * Errors: EINVAL, ESTATE (opt.precond != 0 and no preconditioner built), EDEVICE.
 */
dda_status dda_grad_cext(dda_problem *p, const double *dir_host, const double *pol_host,
                         double *grad_dev, double *cext, dda_stats *stats);

/* Release every device allocation of the handle (NULL is a no-op). */
void dda_destroy(dda_problem *p);

/*
 * Per-kernel timing with HIP events recorded around every launch on the
 * handle's stream.  Enabling resets the counters.  dda_profile_get returns,
 * for kernel kind idx in [0, dda_profile_count()), its name (valid until the
 * handle is destroyed), the number of launches, their summed duration in ms,
 * and the mean algorithmic bytes per launch (read + write, per the traffic
 * model of the kernel; launches of one kind may differ in size).  Only launches that did
 * work are counted: inside a restart cycle whose right-hand sides have all stopped, the
 * cycle's remaining launches return at once, and launches under 2 % of the kind's longest
 * are left out.
 */
dda_status dda_profile_enable(dda_problem *p, int on);
/* Restrict the timing to launches of kernel kind `name` (as dda_profile_get names it), so
 * that the other launches carry no events; NULL or "" times every kind again.  Kinds already
 * collected keep their counts.  EINVAL for a NULL handle. */
dda_status dda_profile_only(dda_problem *p, const char *name);
int dda_profile_count(dda_problem *p);
dda_status dda_profile_get(dda_problem *p, int idx, const char **name, long long *launches,
                           double *total_ms, double *bytes_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* DDA_H */
