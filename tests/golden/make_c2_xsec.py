#!/usr/bin/env python
"""Write ``c2_xsec.txt``: cross sections of the 128^3 benchmark prism computed by the oracle alone.

Test infrastructure.  Calls only ``oracle/`` (and the seeded input generators in ``workloads/``):
the incident field and LDR factor of Sec. 2.1, the zero-padded FFT form of the BTTB product
(Sec. 1 and 2.2), unpreconditioned restarted GMRES (Sec. 4) run far past the benchmark tolerance,
and the Draine-Flatau cross sections (C_sca by the Im G double sum).  Nothing here touches the
GPU library.  The GPU parity test of the same prism compares against the file this writes.

Usage:  python tests/golden/make_c2_xsec.py [--tol 1e-11] [--restart 60] [--workers 8]
Runtime: about half an hour per polarisation on 8 host cores (6.3 million box unknowns).
"""

from __future__ import annotations

import argparse
import datetime
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle import fftmatvec, gmres, physics, system, xsec  # noqa: E402

OUT = os.path.join(HERE, "c2_xsec.txt")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--tol", type=float, default=1e-11)
    ap.add_argument("--restart", type=int, default=60)
    ap.add_argument("--workers", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()

    cfg = w.config_c2()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    t0 = time.time()
    Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d, workers=args.workers)
    print(f"kernel spectrum {time.time() - t0:.1f} s", flush=True)
    rows = []
    for r in range(len(dirs)):
        S = physics.lattice_S(dirs[r], pols[r])
        b = system.incident_field(s.mask, s.k, s.d, dirs[r], pols[r])
        n_mv = [0]

        def mv(x):
            n_mv[0] += 1
            if n_mv[0] % 25 == 0:
                print(f"  wave {r}: {n_mv[0]} products, {time.time() - t0:.0f} s", flush=True)
            return fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh, workers=args.workers)

        c, info = gmres.gmres(mv, b, restart=args.restart, tol=args.tol, maxit=20000)
        res = np.linalg.norm((b - mv(c)).ravel()) / np.linalg.norm(b.ravel())
        ce, ca, cs = xsec.cross_sections(c, s.mask, s.eps, s.k, s.d, dirs[r], pols[r],
                                         workers=args.workers)
        print(f"wave {r}: converged={info['converged']} iters={info['iters']} "
              f"true residual {res:.3e}  C_ext {ce:.15e} C_abs {ca:.3e} C_sca {cs:.15e}", flush=True)
        assert info["converged"], "oracle GMRES did not reach the tolerance"
        rows.append((r, dirs[r], pols[r], info["iters"], res, ce, ca, cs))
    with open(args.out, "w") as fh:
        fh.write("# Cross sections of the 128^3 benchmark prism (hexagonal prism, size parameter 20,\n"
                 "# aspect ratio 1, m = 1.31, plane wave along +z, x and y polarisations), computed by\n"
                 "# the CPU oracle only: oracle.fftmatvec (zero-padded FFT form of the BTTB product,\n"
                 "# Sec. 1 and 2.2), oracle.gmres without preconditioner (restarted GMRES, Sec. 4) to\n"
                 f"# a true relative residual below {args.tol:g}, oracle.xsec (Draine-Flatau forms,\n"
                 "# C_sca by the Im G double sum).  Written by tests/golden/make_c2_xsec.py\n"
                 f"# (restart {args.restart}, {args.workers} workers, {platform.processor() or platform.machine()},\n"
                 f"# {datetime.datetime.now(datetime.timezone.utc).strftime('%Y-%m-%d')}, {time.time() - t0:.0f} s).\n"
                 "# columns: wave dir_x dir_y dir_z pol_x pol_y pol_z iters true_rel_residual "
                 "C_ext C_abs C_sca\n")
        for r, d, p, it, res, ce, ca, cs in rows:
            fh.write(f"{r} {d[0]:.1f} {d[1]:.1f} {d[2]:.1f} {p[0]:.1f} {p[1]:.1f} {p[2]:.1f} {it} "
                     f"{res:.3e} {ce!r} {ca!r} {cs!r}\n")
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
