"""CPU oracle for the preconditioned DDA solve — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct numpy/scipy implementation of what the HIP
path computes, in float64 / complex128, written from the paper (Groth,
Polimeridis & White, "Preconditioning the discrete dipole approximation").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library and never
imports it; the product path must never route through it.

Modules
-------
physics    LDR polarisability (Sec. 2.1) and the dyadic Green tensor (Sec. 2).
system     voxel centres, incident field, the dense DDA matrix (Sec. 2.1-2.2).
fftmatvec  zero-padded FFT convolution form of the BTTB product (Sec. 1, 2.2).
circulant  T. Chan's optimal circulant (eq. Chan), its brute-force Frobenius
           form, and the 2-level block preconditioner (Sec. 3, 3.1).
gmres      restarted right-preconditioned GMRES with Givens rotations (Sec. 4).
xsec       extinction / absorption / scattering cross sections (Draine-Flatau
           forms adapted to the paper's scaling; not in the paper itself).
adjoint    dC_ext/d eps by one adjoint solve (complex-symmetric matrix).
rows       sampled rows of the operator / preconditioner by direct summation,
           for grids too large for anything else.

Each function's docstring names the passage it follows and, where the paper is
silent or garbled, the reading it takes.
"""
