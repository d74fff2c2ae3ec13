#!/usr/bin/env python
"""Benchmark of the preconditioned DDA solve on one MI355X.

One step is the whole hot path for one batch of synthetic input: problem setup (LDR
polarisability, incident field, Green-tensor spectrum by FFT), the 2-level circulant
preconditioner build (Chan generator, FFTs, per-mode block inversion), preconditioned
GMRES(30) for both polarisations to a true relative residual of 1e-5, and the three cross
sections.  Inputs (mask, permittivity) are resident in HBM before timing starts.

Default workload: hexagonal ice prism, aspect ratio 1, size parameter 20, 128^3 voxel grid
(FFT grid 256^3), m = 1.31, plane wave along +z with x and y polarisations, FP64.

Printed: one JSON line with the solve time per step (lower is better), the unpreconditioned
solve for comparison, the FFT matvec throughput, the roofline of the dominant kernel measured
with HIP events on the library's stream during the timed steps, and the CPU oracle timed on
a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DDA solve s to rel. residual 1e-5 (precond vs plain) + FFT-matvec HBM GB/s"
HBM_PEAK_GBPS = 8000.0


def workload(name):
    import workloads as w
    if name == "c1":
        cfg = w.config_c1()
        desc = "hex prism x=2 aspect 1, 16^3 grid (FFT 32^3), m=1.31, +z x-pol, GMRES(30) tol 1e-6"
    else:
        cfg = w.config_c2()
        desc = ("hex prism x=20 aspect 1, 128^3 grid (FFT 256^3), m=1.31, +z x- and y-pol, "
                "GMRES(30) tol 1e-5, 2-level circulant preconditioner")
    return cfg, desc


def operator_bytes(s, nrhs, elem=16):
    """Algorithmic HBM bytes of one FFT matvec (five passes, octant kernel spectrum)."""
    nz, ny, nx = s.shape
    N = nx * ny * nz
    e = elem
    p1 = 16 * 3 * N + N + e * 6 * N
    p2 = e * (6 * N + 12 * N)
    p3 = e * 24 * N
    p4 = e * (12 * N + 6 * N)
    p5 = e * 6 * N + 16 * 3 * N + N + 16 * 3 * N + 16 * N
    return nrhs * (p1 + p2 + p3 + p4 + p5) + e * 6 * (nx + 1) * (ny + 1) * (nz + 1)


def gemv_algorithmic_bytes(s, nrhs, elem=16):
    """Algorithmic bytes of one block-product launch: the symmetric-packed inverse blocks,
    l m (3n)^2 s / 16 (n the dense level's extent: the occupied z layers), and the mode vectors
    read and written once, 2 * 3N * s per right-hand side."""
    nz, ny, nx = s.shape
    occ = s.mask.reshape(nz, -1).any(axis=1)
    n = int(occ.nonzero()[0][-1] - occ.nonzero()[0][0] + 1)
    return nx * ny * (3 * n) ** 2 * elem / 16.0 + nrhs * 2.0 * 3 * nx * ny * nz * elem


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_hex128_fp64.txt")
GOLDEN_C2 = os.path.join(ROOT, "tests", "golden", "c2_xsec.txt")


def golden_deviation(cext, csca):
    """Relative deviation of the step's cross sections (solved to the workload's tolerance)
    from the oracle-only reference solved to 1e-11, per wave; None without the file."""
    if not os.path.exists(GOLDEN_C2):
        return None
    rows = [ln.split() for ln in open(GOLDEN_C2) if ln.strip() and not ln.startswith("#")]
    out = {}
    for f in rows:
        r = int(f[0])
        if r < len(cext):
            out[f"wave{r}"] = dict(cext=abs(cext[r] - float(f[9])) / float(f[9]),
                                   csca=abs(csca[r] - float(f[11])) / float(f[11]))
    return out


def source_digest():
    """Digest of the HIP sources; counter figures taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1903_09802_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a plain copy kernel), or
    None when there is none for this kernel or it was taken on other sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest, rows = None, {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) >= 2 and f[0] == "source_digest:":
                digest = f[1]
            elif len(f) >= 6 and f[0] == "kernel" and f[2] == "fetch_bytes" and f[4] == "write_bytes":
                rows[f[1]] = float(f[3]) + float(f[5])
    if digest != source_digest():
        return None
    return rows.get(kernel)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(cfg, plain_iters, restart=30, k_it=8):
    """The oracle timed on a fixed, bounded piece of the same workload, scaled to one solve.

    Timed oracle calls, all with the real 128^3 operator: the kernel spectrum (scipy FFTs of
    the padded Green tensor), one FFT matvec, and ``k_it`` iterations of the oracle's own
    restarted GMRES (FFT matvec + modified Gram-Schmidt) on the first wave.  The oracle's
    preconditioner would need all 16,384 dense 384^2 mode blocks (38.7 GB), so its step is
    quoted for its plain GMRES to the same tolerance: the spectrum once, then per wave the
    iteration count the GPU's plain solve took, each iteration one matvec plus the Gram-Schmidt
    projections of its position in the cycle, and one residual matvec per cycle.
    """
    import numpy as np
    import scipy.fft as sfft

    from oracle import fftmatvec, gmres, physics, system

    cores = len(os.sched_getaffinity(0))
    s = cfg["scatterer"]
    dirs, pols = cfg["dirs"], cfg["pols"]
    with sfft.set_workers(cores):
        t0 = time.perf_counter()
        Kh = fftmatvec.kernel_padded_fft(s.shape, s.k, s.d, workers=cores)
        t_setup = time.perf_counter() - t0
        S = physics.lattice_S(dirs[0], pols[0])
        b = system.incident_field(s.mask, s.k, s.d, dirs[0], pols[0])

        def mv(x):
            return fftmatvec.fft_matvec(x, s.mask, s.eps, s.k, s.d, S, Khat=Kh, workers=cores)

        mv(b)  # first call: FFT plans
        t0 = time.perf_counter()
        mv(b)
        t_mv = time.perf_counter() - t0
        t0 = time.perf_counter()
        gmres.gmres(mv, b, restart=restart, tol=0.0, maxit=k_it)
        t_run = time.perf_counter() - t0
    # k_it iterations hold k_it + 2 matvecs (initial and final residual) and k_it (k_it + 1) / 2
    # projections (dot + update each)
    t_proj = max(0.0, t_run - (k_it + 2) * t_mv) / (k_it * (k_it + 1) / 2)
    per_wave = []
    for it in plain_iters:
        cycles = -(-it // restart)
        proj = sum((j % restart) + 1 for j in range(it))
        per_wave.append((it + cycles + 1) * t_mv + proj * t_proj)
    est = t_setup + sum(per_wave)
    sample = (f"oracle (numpy/scipy, complex128) on {cores} host cores ({cpu_model()}): kernel "
              f"spectrum of the 128^3 prism, one FFT matvec and {k_it} iterations of the oracle's "
              f"GMRES({restart}) with the real operator, timed; quoted for its plain GMRES solve of "
              f"both waves to the same tolerance ({'+'.join(str(i) for i in plain_iters)} "
              f"iterations, the GPU's plain counts), since its preconditioner needs 38.7 GB of blocks")
    return dict(value=est, unit="s", cores=cores, kind="oracle", sample=sample, cpu=cpu_model(),
                parts=dict(setup_s=t_setup, matvec_s=t_mv, gs_projection_s=t_proj,
                           gmres_iteration_s=(t_run - 2 * t_mv) / k_it, timed_s=t_setup + 2 * t_mv + t_run))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "c3study", "c4", "c5", "plates", "axes", "levels",
                             "alpha"],
                    help="c2 (default): the 128^3 step; c1: solve latency at 16^3; c3: FP32-refined vs "
                         "FP64 at 256^3; c4: batched prisms; c5: adjoint gradient; the rest: studies")
    ap.add_argument("--c3-case", type=int, default=0, help="c3: 0 -> m = 1.31+0.001i, 1 -> m = 1.78")
    ap.add_argument("--c3-variants", default="gmres30,gmres100,gmres300,bicgstab,gmres100_xdense",
                    help="c3study: comma-separated solver variants")
    ap.add_argument("--c4-prisms", type=int, default=16)
    ap.add_argument("--c4-chunk", type=int, default=32, help="c4: right-hand sides per batched solve")
    ap.add_argument("--c4-precision", type=int, default=0, help="c4: 0 FP64, 1 FP32 inside FP64 refinement")
    ap.add_argument("--c4-compare", type=int, default=0,
                    help="c4: after the timed batch, solve the first N waves of every prism one per "
                         "solve in FP64 and compare their cross sections and rate with the batch's")
    ap.add_argument("--c4-streams", type=int, default=1,
                    help="c4: prisms in flight at once, each on its own stream (worker threads)")
    ap.add_argument("--plates", default="0.1:1.2",
                    help="plates: 'all', or L/a[:mu[:x,x,...]] (e.g. 0.1, 0.2:1.4, 0.1:2.0:10,20)")
    ap.add_argument("--plates-plain", action="store_true",
                    help="plates: also run the unpreconditioned solvers")
    ap.add_argument("--plates-plain-max-x", type=float, default=1e9,
                    help="plates: run the unpreconditioned solvers only up to this size parameter")
    ap.add_argument("--plates-left", action="store_true",
                    help="plates: also run preconditioned GMRES with left preconditioning (the "
                         "paper's P^-1 A x = P^-1 b, stopping on the preconditioned residual)")
    ap.add_argument("--plates-restart", type=int, default=500,
                    help="plates: GMRES restart length (500 keeps the whole Krylov space for every "
                         "case the paper's unrestarted GMRES solved)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-bicgstab", action="store_true",
                    help="skip the preconditioned BiCGStab solve reported beside the GMRES step")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB elementwise copy kernel (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the solver has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1903_09802_amd.dda import Problem, load

    load()
    if args.workload == "c1":
        return bench_c1(args)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c3study":
        return bench_c3_study(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "plates":
        return bench_plates(args)
    if args.workload == "axes":
        return bench_axes(args)
    if args.workload == "alpha":
        bench_alpha(args)
        return
    if args.workload == "levels":
        return bench_levels(args)
    cfg, desc = workload(args.workload)
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    nrhs = len(dirs)
    tol = cfg["tol"]
    mask = torch.from_numpy(s.mask).cuda()
    eps = torch.from_numpy(s.eps).cuda()
    torch.cuda.synchronize()

    def step(profile=False, graph=True, only=None):
        prob = Problem(mask, eps, s.k, s.d, precond=2, tol=tol, restart=30, max_rhs=nrhs,
                       graph=graph)
        if profile:
            prob.profile_enable(True)
            prob.profile_only(only)
        prob.build_preconditioner(0.0)
        out = prob.solve(dirs, pols, return_c=False, xsec=True)
        prof = prob.profile() if profile else None
        prob.close()
        return out, prof

    def aggregate(profs):
        # per-kernel totals (HIP events on the library stream), largest total first
        agg = {}
        for pr in profs:
            for k in pr:
                a = agg.setdefault(k["name"], dict(launches=0, total_ms=0.0, total_bytes=0.0))
                a["launches"] += k["launches"]
                a["total_ms"] += k["total_ms"]
                a["total_bytes"] += k["bytes_per_launch"] * k["launches"]
        for a in agg.values():
            a["bytes"] = a["total_bytes"] / max(1, a["launches"])
        return sorted(((k, v) for k, v in agg.items() if v["launches"]), key=lambda kv: -kv[1]["total_ms"])

    def dominant(kernels):
        # the streaming kernel with the largest total (setup kernels excluded)
        return [kv for kv in kernels if not kv[0].startswith(
            ("pc_gj", "pc_sweep", "pc_assemble", "fft_rows_setup", "fft_strided_setup"))][0]

    # the last warmup step times every kernel (untimed): the per-kernel table and the dominant
    # kernel, which the timed steps then time alone, so that the other launches carry no events
    full = None
    for w in range(args.warmup):
        _, pr = step(profile=w == args.warmup - 1)
        full = pr or full
    only = dominant(aggregate([full]))[0] if full else None
    torch.cuda.synchronize()
    outs, profs = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        o, pr = step(profile=True, only=only)
        outs.append(o)
        profs.append(pr)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1000.0 * elapsed / args.steps
    last = outs[-1]
    p_iters = [st["iters"] for st in last["stats"]]
    p_res = [st["rel_residual"] for st in last["stats"]]
    converged = all(st["converged"] for st in last["stats"])

    kernels = aggregate([full]) if full else aggregate(profs)
    dom_name, dom = dominant(aggregate(profs))
    avg_ms = dom["total_ms"] / max(1, dom["launches"])
    # algorithmic bytes per launch: the traffic model of each pass (the library's figures), except
    # the block product, whose stored layout (full diagonal tiles, (l/2+1)(m/2+1) modes) holds more
    # than the packed count l m (3n)^2 s / 16 it is judged by
    alg = gemv_algorithmic_bytes(s, nrhs) if dom_name == "pc_gemv_f64" else dom["bytes"]
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom_name)
    roofline = dict(bound="hbm", kernel=dom_name, achieved=achieved, peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBPS, traffic=traffic, avg_launch_ms=avg_ms,
                    algorithmic_bytes_per_launch=alg, layout_bytes_per_launch=dom["bytes"],
                    traffic_over_algorithmic=(traffic / alg) if traffic else None)
    # per-kernel table: the fully timed warmup step (one step), else the timed steps
    all_ms = sum(v["total_ms"] for _, v in kernels)
    kernel_table = {k: dict(launches=v["launches"], avg_ms=v["total_ms"] / max(1, v["launches"]),
                            share=v["total_ms"] / max(1e-12, all_ms),
                            GBps=(v["bytes"] / (v["total_ms"] / max(1, v["launches"]) * 1e-3) / 1e9)
                            if v["total_ms"] > 0 else None)
                    for k, v in kernels[:14]}

    # the same step without per-kernel events: restart cycles replayed from HIP graphs, and
    # launched one by one
    unprofiled = {}
    for graph in (True, False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            step(profile=False, graph=graph)
        torch.cuda.synchronize()
        unprofiled["graph" if graph else "eager"] = (time.perf_counter() - t0) / 3

    # matvec throughput (FP64, both RHS) and preconditioner apply
    prob = Problem(mask, eps, s.k, s.d, precond=2, tol=tol, restart=30, max_rhs=nrhs)
    prob.build_preconditioner(0.0)
    x = torch.randn((nrhs, 3) + s.shape, dtype=torch.complex128, device="cuda") * mask
    y = torch.empty_like(x)
    prob.apply_operator(x, dirs, pols, out=y)
    prob.apply_preconditioner(x, out=y)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.apply_operator(x, dirs, pols, out=y)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.apply_preconditioner(x, out=y)
    torch.cuda.synchronize()
    t_pc = (time.perf_counter() - t0) / reps
    mv_bytes = operator_bytes(s, nrhs)
    matvec_gbps = mv_bytes / t_mv / 1e9
    # plain GMRES for comparison (same problem, no preconditioner)
    plain = None
    if not args.no_plain:
        pp = Problem(mask, eps, s.k, s.d, precond=0, tol=tol, restart=30, max_rhs=nrhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = pp.solve(dirs, pols, return_c=False, xsec=True)
        torch.cuda.synchronize()
        plain = dict(solve_s=time.perf_counter() - t0, iters=[st["iters"] for st in o["stats"]],
                     converged=all(st["converged"] for st in o["stats"]),
                     cext=o["cext"].tolist())
        pp.close()
    # preconditioned BiCGStab on the same problem (the paper's second solver, cap 4000)
    bicg = None
    if not args.no_bicgstab:
        pb = Problem(mask, eps, s.k, s.d, precond=2, tol=tol, restart=30, max_rhs=nrhs,
                     max_iter=4000, solver="bicgstab")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.build_preconditioner(0.0)
        o = pb.solve(dirs, pols, return_c=False, xsec=True)
        torch.cuda.synchronize()
        bicg = dict(step_s=time.perf_counter() - t0, iters=[st["iters"] for st in o["stats"]],
                    restarts=[max(0, st["cycles"] - 1) for st in o["stats"]],
                    converged=all(st["converged"] for st in o["stats"]),
                    rel_residual=[st["rel_residual"] for st in o["stats"]],
                    cext=o["cext"].tolist())
        pb.close()
    prob.close()

    if args.copy_probe:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB: the scale for HBM byte counters
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, plain["iters"] if plain else [197] * nrhs)

    line = dict(
        metric=METRIC, value=ms / 1000.0, unit="s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms, higher_is_better=False, scaling="weak", vs_baseline=None, dtype="f64",
        data="synthetic",
        config=dict(workload=desc, grid=list(s.shape), n_occupied=int(s.n_occ), nrhs=nrhs,
                    size_parameter=s.meta.get("x"), restart=30, tol=tol),
        precond_iters=p_iters, precond_rel_residual=p_res, converged=converged,
        phases_ms=dict(create=1e3 * last["stats"][0]["t_setup"], build=1e3 * last["stats"][0]["t_build"],
                       solve=1e3 * last["stats"][0]["t_solve"]),
        cext=last["cext"].tolist(), cabs=last["cabs"].tolist(), csca=last["csca"].tolist(),
        xsec_rel_dev_vs_oracle_golden=golden_deviation(last["cext"].tolist(), last["csca"].tolist()),
        step_s_unprofiled=unprofiled, plain=plain, bicgstab=bicg, matvec_ms=1000 * t_mv, matvec_GBps=matvec_gbps,
        matvec_frac_hbm=matvec_gbps / HBM_PEAK_GBPS, precond_apply_ms=1000 * t_pc,
        roofline=roofline, kernels=kernel_table, cpu_baseline=cpu,
    )
    print(json.dumps(line), flush=True)


def _emit(line):
    print(json.dumps(line), flush=True)


def bench_c1(args):
    """Latency: the 16^3 prism (x = 2) to 1e-6, preconditioned and plain, with restart cycles
    replayed from HIP graphs and launched one by one; median of 7 solves after a warm one."""
    import numpy as np
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cfg = w.config_c1()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    mask = torch.from_numpy(s.mask).cuda()
    eps = torch.from_numpy(s.eps).cuda()
    res = {}
    for precond in (2, 0):
        for graph in (True, False):
            prob = Problem(mask, eps, s.k, s.d, precond=precond, tol=cfg["tol"], restart=30, graph=graph)
            if precond:
                prob.build_preconditioner(0.0)
            prob.solve(dirs, pols, return_c=False, xsec=False)
            times = []
            for _ in range(7):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = prob.solve(dirs, pols, return_c=False, xsec=False)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            st = out["stats"][0]
            t = float(np.median(times))
            res[f"{'precond' if precond else 'plain'}_{'graph' if graph else 'eager'}"] = dict(
                solve_ms=1e3 * t, iters=st["iters"], cycles=st["cycles"], per_iter_us=1e6 * t / max(1, st["iters"]),
                setup_ms=1e3 * st["t_setup"], build_ms=1e3 * st["t_build"], converged=st["converged"])
            prob.close()
    _emit(dict(metric="DDA solve latency, 16^3 prism to 1e-6", workload="c1", unit="ms",
               value=res["precond_graph"]["solve_ms"], higher_is_better=False,
               config=dict(workload="hex prism x=2 aspect 1, 16^3 grid (FFT 32^3), m=1.31, +z x-pol, "
                           "GMRES(30) tol 1e-6", grid=list(s.shape), n_occupied=int(s.n_occ)),
               results=res, dtype="f64", data="synthetic"))


def bench_c3(args):
    """Precision: FP32 operator and preconditioner inside FP64 refinement vs all-FP64, 256^3."""
    import numpy as np
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cfg = w.config_c3(args.c3_case)
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    mask = torch.from_numpy(s.mask).cuda()
    eps = torch.from_numpy(s.eps).cuda()
    res = {}
    for precision in (1, 0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = Problem(mask, eps, s.k, s.d, precond=2, tol=cfg["tol"], restart=30, precision=precision)
        t1 = time.perf_counter()
        prob.build_preconditioner(0.0)
        t2 = time.perf_counter()
        out = prob.solve(dirs, pols, return_c=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        prob.close()
        del prob
        torch.cuda.empty_cache()
        st = out["stats"][0]
        res[precision] = dict(setup_s=t1 - t0, build_s=t2 - t1, solve_s=t3 - t2, total_s=t3 - t0,
                              iters=st["iters"], refinements=st["refinements"],
                              rel_residual=st["rel_residual"], converged=st["converged"],
                              cext=float(out["cext"][0]), cabs=float(out["cabs"][0]),
                              csca=float(out["csca"][0]))
    dev = {k: abs(res[1][k] - res[0][k]) / abs(res[0][k]) for k in ("cext", "csca")}
    _emit(dict(metric=METRIC, workload="c3", unit="s", value=res[1]["total_s"], higher_is_better=False,
               config=dict(workload=f"hex prism x=40 aspect 2, 256^3 grid (FFT 512^3), m="
                           f"{'1.31+0.001i' if args.c3_case == 0 else '1.78'}, +z x-pol, tol 1e-5",
                           grid=list(s.shape), n_occupied=int(s.n_occ)),
               fp32_refined=res[1], fp64=res[0], speedup_fp32=res[0]["total_s"] / res[1]["total_s"],
               xsec_rel_dev_fp32_vs_fp64=dev, dtype="f32 inner / f64 outer", data="synthetic"))


def bench_c3_study(args):
    """The 256^3 prism (m = 1.78 by default): which solver settings converge.  One line per
    variant: GMRES(m) for several m, BiCGStab, the other dense axis, FP32-refined."""
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cfg = w.config_c3(args.c3_case)
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    mask = torch.from_numpy(s.mask).cuda()
    eps = torch.from_numpy(s.eps).cuda()
    variants = {
        "gmres30": dict(restart=30), "gmres100": dict(restart=100), "gmres300": dict(restart=300),
        "bicgstab": dict(solver="bicgstab", restart=30, max_iter=4000),
        "gmres100_xdense": dict(restart=100, dense_axis=0),
        "gmres300_fp32": dict(restart=300, precision=1),
        # close to the paper's unrestarted GMRES (its Sec. 4 cap is 2000 iterations): 1000
        # Krylov vectors of the 256^3 prism take 130 GB in FP64
        "gmres1000": dict(restart=1000), "gmres1000_left": dict(restart=1000, precond_side="left"),
    }
    for name in args.c3_variants.split(","):
        kw = dict(precond=2, tol=cfg["tol"], max_iter=2000)
        kw.update(variants[name])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = Problem(mask, eps, s.k, s.d, **kw)
        prob.build_preconditioner(0.0)
        t1 = time.perf_counter()
        out = prob.solve(dirs, pols, return_c=False, history=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        prob.close()
        del prob
        torch.cuda.empty_cache()
        st = out["stats"][0]
        h = st.pop("history")
        _emit(dict(workload="c3_study", case=args.c3_case, variant=name, options=kw,
                   build_s=t1 - t0, solve_s=t2 - t1, iters=st["iters"], cycles=st["cycles"],
                   converged=st["converged"], rel_residual=st["rel_residual"],
                   history_every_100=[float(v) for v in h[::100]], history_min=float(h.min()) if len(h) else None,
                   cext=float(out["cext"][0]), csca=float(out["csca"][0]), cabs=float(out["cabs"][0])))


def bench_c4(args):
    """Batching: seeded prisms of uneven grids, 128 waves each, solved in RHS blocks.

    With --c4-streams S > 1, S worker threads each take the next prism and run it on a stream of
    their own (the library releases the interpreter lock in every call), so prisms overlap on
    the GPU.  Latency is per prism from the start of its work to its last converged wave."""
    import threading

    import numpy as np
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem, lattice_factor

    cfg = w.config_c4(n_prisms=args.c4_prisms)
    prisms = list(enumerate(cfg["prisms"]))
    # the largest grids first, so that a worker finishing early takes the small ones
    prisms.sort(key=lambda ip: -ip[1]["scatterer"].mask.size)
    lock = threading.Lock()
    lat, solved, iters, errors = {}, [0], [], []
    first = {}  # prism -> (C_ext, C_sca) of its first waves in the batch, for --c4-compare

    def run(pr, stream):
        s, dirs, pols = pr["scatterer"], pr["dirs"], pr["pols"]
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            mask = torch.from_numpy(s.mask).cuda()
            eps = torch.from_numpy(s.eps).cuda()
            stream.synchronize()
            chunk = args.c4_chunk
            prob = Problem(mask, eps, s.k, s.d, precond=2, tol=cfg["tol"], restart=30,
                           precision=args.c4_precision, max_rhs=chunk, stream=stream)
            prob.build_preconditioner(lattice_factor(dirs, pols)[1])
            conv, its = 0, []
            for q0 in range(0, len(dirs), chunk):
                out = prob.solve(dirs[q0:q0 + chunk], pols[q0:q0 + chunk], return_c=False)
                conv += sum(st["converged"] for st in out["stats"])
                its += [st["iters"] for st in out["stats"]]
                if q0 == 0:
                    ce, cs = out["cext"].copy(), out["csca"].copy()
            stream.synchronize()
            prob.close()
        return time.perf_counter() - t0, conv, its, (ce, cs)

    def worker():
        stream = torch.cuda.Stream()
        while True:
            with lock:
                if not prisms or errors:
                    return
                i, pr = prisms.pop(0)
            try:
                t, conv, its, xs = run(pr, stream)
            except Exception as e:  # reported after the join
                with lock:
                    errors.append(e)
                return
            with lock:
                lat[i] = t
                first[i] = xs
                solved[0] += conv
                iters.extend(its)
                print(f"c4 prism {i} grid {pr['scatterer'].nx}^3: {t:.3f} s ({len(lat)}/{len(cfg['prisms'])})",
                      file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t_all = time.perf_counter()
    threads = [threading.Thread(target=worker) for _ in range(max(1, args.c4_streams))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    if errors:
        raise errors[0]
    lat = [lat[i] for i in sorted(lat)]
    n_rhs = sum(len(pr["dirs"]) for pr in cfg["prisms"])
    compare = None
    if args.c4_compare > 0:
        # the plain FP64 path: the same waves one per solve (solve time only; the batch's rate
        # includes each prism's setup and build), against the batch's cross sections
        K = args.c4_compare
        dev_e, dev_s, t1, n1, its1 = [], [], 0.0, 0, []
        for i, pr in enumerate(cfg["prisms"]):
            s, dirs, pols = pr["scatterer"], pr["dirs"], pr["pols"]
            prob = Problem(torch.from_numpy(s.mask).cuda(), torch.from_numpy(s.eps).cuda(), s.k, s.d,
                           precond=2, tol=cfg["tol"], restart=30, precision=0, max_rhs=1)
            prob.build_preconditioner(lattice_factor(dirs, pols)[1])
            torch.cuda.synchronize()
            for q in range(min(K, len(dirs))):
                t0 = time.perf_counter()
                out = prob.solve(dirs[q:q + 1], pols[q:q + 1], return_c=False)
                t1 += time.perf_counter() - t0
                n1 += 1
                its1.append(out["stats"][0]["iters"])
                dev_e.append(abs(first[i][0][q] - out["cext"][0]) / abs(out["cext"][0]))
                dev_s.append(abs(first[i][1][q] - out["csca"][0]) / abs(out["csca"][0]))
            prob.close()
        compare = dict(waves_per_prism=K, single_fp64_solves_per_s_solve_only=n1 / t1,
                       single_iters_mean=float(np.mean(its1)),
                       max_rel_dev_cext=float(np.max(dev_e)), max_rel_dev_csca=float(np.max(dev_s)))
    _emit(dict(metric="RHS solves/s (batched, to rel. residual 1e-5)", workload="c4",
               value=n_rhs / total, unit="solves/s", higher_is_better=True,
               prisms_per_s=len(lat) / total, total_s=total, rhs_total=n_rhs, rhs_converged=solved[0],
               latency_p50_s=float(np.percentile(lat, 50)), latency_p99_s=float(np.percentile(lat, 99)),
               iters_mean=float(np.mean(iters)), iters_max=int(np.max(iters)),
               grids=[pr["scatterer"].nx for pr in cfg["prisms"]], rhs_chunk=args.c4_chunk,
               streams=args.c4_streams, vs_single_fp64=compare,
               dtype="f64" if args.c4_precision == 0 else "f32 inner / f64 outer", data="synthetic"))


def bench_c5(args):
    """Differentiation: adjoint dC_ext/d eps on the 64^3 jittered prism vs a forward solve."""
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cfg = w.config_c5()
    s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
    mask = torch.from_numpy(s.mask).cuda()
    eps = torch.from_numpy(s.eps).cuda()
    prob = Problem(mask, eps, s.k, s.d, precond=2, tol=cfg["tol"], restart=30)
    prob.build_preconditioner(0.0)
    prob.solve(dirs, pols, return_c=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd = prob.solve(dirs, pols, return_c=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, cext, stats, status = prob.grad_cext(dirs[0], pols[0])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prob.close()
    _emit(dict(metric="adjoint gradient s (forward + adjoint solve)", workload="c5",
               value=t2 - t1, unit="s", higher_is_better=False, forward_s=t1 - t0,
               grad_over_forward=(t2 - t1) / (t1 - t0), cext=cext, iters=[st["iters"] for st in stats],
               grad_norm=float(torch.linalg.vector_norm(g).item()), dtype="f64", data="synthetic",
               config=dict(workload="hex prism x=10 aspect 1, 64^3 grid, eps = 1.7161(1+U[-0.05,0.05])",
                           grid=list(s.shape), n_occupied=int(s.n_occ))))


PAPER_TABLES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                            "paper_tables_3_4.txt")


def paper_tables():
    """{(l_over_a, mu, x): row} from the transcription of the paper's Tables 3 and 4."""
    keys = ("total", "plain_gmres_its", "plain_gmres_s", "plain_bicg_its", "plain_bicg_s",
            "build_s", "prec_gmres_its", "prec_gmres_s", "prec_bicg_its", "prec_bicg_s")
    out = {}
    for ln in open(PAPER_TABLES):
        f = ln.split()
        if not f or f[0].startswith("#"):
            continue
        vals = [v if v in ("nc", "oom") else float(v) for v in f[3:13]]
        out[(float(f[0]), float(f[1]), int(f[2]))] = dict(zip(keys, vals), table=f[13])
    return out


def _plate_cases(spec):
    import workloads as w
    tab = paper_tables()
    if spec == "all":
        return sorted(tab)
    parts = spec.split(":")
    la = float(parts[0])
    mus = [float(parts[1])] if len(parts) > 1 else list(w.PLATE_MU)
    xs = [int(v) for v in parts[2].split(",")] if len(parts) > 2 else list(w.PLATE_X)
    return [(la, mu, x) for mu in mus for x in xs if (la, mu, x) in tab]


def bench_plates(args):
    """The paper's Sec. 4 plate sweep: preconditioned (and optionally plain) GMRES(m) and
    BiCGStab to 1e-5 per case, one JSON line each, beside the paper's Tables 3-4 entries."""
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import DDAError, Problem

    tab = paper_tables()
    for la, mu, x in _plate_cases(args.plates):
        rounding = w.plate_fit_rounding(la, mu, x, tab[(la, mu, x)]["total"])
        cfg = w.plate_case(la, mu, x, rounding=rounding)
        s, dirs, pols = cfg["scatterer"], cfg["dirs"], cfg["pols"]
        line = dict(workload="plates", l_over_a=la, mu=mu, x=x, restart=args.plates_restart,
                    rounding=rounding,
                    grid=list(s.shape),
                    fit_grid=list(s.meta["fit_shape"]), total_voxels=int(s.meta["fit_total"]),
                    n_occupied=int(s.n_occ), paper=tab[(la, mu, x)])
        if max(s.shape) > 512:
            line["skipped"] = "grid dimension above 512"
            _emit(line)
            continue
        mask = torch.from_numpy(s.mask).cuda()
        eps = torch.from_numpy(s.eps).cuda()
        plain = args.plates_plain and x <= args.plates_plain_max_x
        runs = [("prec", 2)] + ([("plain", 0)] if plain else [])
        try:
            for tag, pc in runs:
                res = {}
                solvers = [("gmres", "gmres", 2000, "right"), ("bicgstab", "bicgstab", 4000, "right")]
                if pc and args.plates_left:
                    # the paper's side: GMRES on P^-1 A x = P^-1 b, stopping on the
                    # preconditioned residual
                    solvers.append(("gmres_left", "gmres", 2000, "left"))
                for key, solver, cap, side in solvers:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    prob = Problem(mask, eps, s.k, s.d, precond=pc, tol=cfg["tol"],
                                   restart=args.plates_restart if solver == "gmres" else 30,
                                   max_iter=cap, solver=solver, precond_side=side)
                    try:
                        torch.cuda.synchronize()
                        t1 = time.perf_counter()
                        if pc:
                            prob.build_preconditioner(0.0)
                        torch.cuda.synchronize()
                        t2 = time.perf_counter()
                        o = prob.solve(dirs, pols, return_c=False, xsec=True)
                        torch.cuda.synchronize()
                        t3 = time.perf_counter()
                    finally:
                        prob.close()
                    st = o["stats"][0]
                    res[key] = dict(its=st["iters"], converged=bool(st["converged"]),
                                       rel_residual=st["rel_residual"], setup_s=t1 - t0,
                                       build_s=(t2 - t1) if pc else None, solve_s=t3 - t2,
                                       cext=float(o["cext"][0]))
                line[tag] = res
        except DDAError as e:
            line["error"] = str(e)
        del mask, eps
        torch.cuda.empty_cache()
        _emit(line)


def bench_axes(args):
    """Choice of circulant axes (option dense_axis) on elongated prisms (axis along z): the
    paper's layout keeps the long axis dense; the alternative makes it a circulant level."""
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cases = [("prism x=20 aspect 2, 128^3, m=1.31", w.hex_prism_grid(20.0, 2.0, 128, 1.31)),
             ("prism x=20 aspect 4, 128^3, m=1.31", w.hex_prism_grid(20.0, 4.0, 128, 1.31)),
             ("prism x=20 aspect 2, 128^3, m=1.78", w.hex_prism_grid(20.0, 2.0, 128, 1.78))]
    dirs, pols = w.plane_wave_z(("x",))
    for desc, s in cases:
        mask = torch.from_numpy(s.mask).cuda()
        eps = torch.from_numpy(s.eps).cuda()
        for axis in (2, 0):
            line = dict(workload="axes", case=desc, grid=list(s.shape), n_occupied=int(s.n_occ),
                        dense_axis=axis)
            for solver, cap in (("gmres", 2000), ("bicgstab", 4000)):
                prob = Problem(mask, eps, s.k, s.d, precond=2, tol=1e-5, restart=30, max_iter=cap,
                               solver=solver, dense_axis=axis)
                try:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    prob.build_preconditioner(0.0)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    o = prob.solve(dirs, pols, return_c=False, xsec=True)
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                finally:
                    prob.close()
                st = o["stats"][0]
                line[solver] = dict(its=st["iters"], converged=bool(st["converged"]),
                                    build_s=t1 - t0, solve_s=t2 - t1, cext=float(o["cext"][0]))
            _emit(line)
        del mask, eps
        torch.cuda.empty_cache()


def bench_levels(args):
    """1-level vs 2-level circulant preconditioner on needles (long axis z): the 1-level one
    is circulant along the needle (dense_axis = 1 puts z on the circulant x level) with dense
    (3 nx ny)^2 blocks; the 2-level one keeps z dense."""
    import numpy as np
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    cases = [("needle 12x12x256, m=1.31", w.cuboid_grid(12, 12, 256, 2.0, 0.25, 1.31)),
             ("needle 16x16x256, m=1.31", w.cuboid_grid(16, 16, 256, 2.0, 0.25, 1.31)),
             ("needle 12x12x256, m=1.78", w.cuboid_grid(12, 12, 256, 2.0, 0.25, 1.78))]
    dirs, pols = np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 0.0, 1.0]])
    for desc, s in cases:
        mask = torch.from_numpy(s.mask).cuda()
        eps = torch.from_numpy(s.eps).cuda()
        for precond, axis in ((0, 2), (2, 2), (1, 1)):
            line = dict(workload="levels", case=desc, grid=list(s.shape), precond=precond,
                        dense_axis=axis)
            prob = Problem(mask, eps, s.k, s.d, precond=precond, tol=1e-5, restart=30,
                           max_iter=2000, dense_axis=axis)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if precond:
                    prob.build_preconditioner(0.0)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = prob.solve(dirs, pols, return_c=False, xsec=True)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
            finally:
                prob.close()
            st = o["stats"][0]
            line.update(its=st["iters"], converged=bool(st["converged"]), build_s=t1 - t0,
                        solve_s=t2 - t1, cext=float(o["cext"][0]))
            _emit(line)
        del mask, eps
        torch.cuda.empty_cache()


def bench_alpha(args):
    """Readings of the preconditioner's constant diagonal (option alpha_avg) on inhomogeneous
    prisms: 1/alpha of the mean permittivity, the mean of 1/alpha, and the paper's modal value
    over the body; and the circulant-plus-diagonal preconditioner (option diag_steps) around
    the first two.  GMRES(30) to 1e-5, one wave (+z, x-pol)."""
    import numpy as np
    import torch

    import workloads as w
    from paper_1903_09802_amd.dda import Problem

    def inclusions(x, grid, m_host, m_inc, frac, seed):
        s = w.hex_prism_grid(x, 1.0, grid, m_host)
        occ = s.mask.astype(bool)
        rng = np.random.default_rng(seed)
        pick = occ & (rng.random(s.mask.shape) < frac)
        s.eps = np.where(pick, m_inc ** 2, s.eps).astype(np.complex128)
        return s

    def core(x, grid, m_host, m_core, r_frac):
        s = w.hex_prism_grid(x, 1.0, grid, m_host)
        nz, ny, nx = s.shape
        zz, yy, xx = np.meshgrid(*(np.arange(n) - (n - 1) / 2 for n in s.shape), indexing="ij")
        inner = (xx / (nx / 2)) ** 2 + (yy / (ny / 2)) ** 2 + (zz / (nz / 2)) ** 2 < r_frac ** 2
        s.eps = np.where(s.mask.astype(bool) & inner, m_core ** 2, s.eps).astype(np.complex128)
        return s

    cases = [("prism x=20 128^3, ice m=1.31 with 30% random voxels at m=1.78",
              inclusions(20.0, 128, 1.31, 1.78, 0.30, 7)),
             ("prism x=20 128^3, ice m=1.31 with a m=1.5 core (radius 0.6)",
              core(20.0, 128, 1.31, 1.5, 0.6)),
             ("prism x=10 64^3, eps 1.7161 (1 + U[-0.05, 0.05])", w.config_c5()["scatterer"])]
    dirs, pols = w.plane_wave_z(("x",))
    for desc, s in cases:
        mask = torch.from_numpy(s.mask).cuda()
        eps = torch.from_numpy(s.eps).cuda()
        runs = [(a, 0) for a in ("mean_eps", "mean_alpha", "mode")]
        runs += [(a, k) for a in ("mean_eps", "mean_alpha") for k in (1, 2, 4)]
        for avg, steps in runs:
            line = dict(workload="alpha", case=desc, grid=list(s.shape), alpha_avg=avg,
                        diag_steps=steps)
            prob = Problem(mask, eps, s.k, s.d, precond=2, tol=1e-5, restart=30, max_iter=2000,
                           alpha_avg=avg, diag_steps=steps)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                prob.build_preconditioner(0.0)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = prob.solve(dirs, pols, return_c=False, xsec=True)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
            finally:
                prob.close()
            st = o["stats"][0]
            line.update(its=st["iters"], converged=bool(st["converged"]), build_s=t1 - t0,
                        solve_s=t2 - t1, cext=float(o["cext"][0]))
            _emit(line)
        del mask, eps
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
