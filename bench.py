#!/usr/bin/env python3
"""Benchmark of the WaveHoltz hot path on one MI355X.

Workload (default): the 512^3 unit cube, 2nd-order 7-point stencil, c = 1 with
a random ball of c = 1.5, omega = 80, point-like Gaussian source; FP32 state
and stencil arithmetic with the filter accumulation and the Krylov vectors in
FP64, 4 leapfrog steps per pass over HBM.  One step = a fixed block of
--iters (default 100) conjugate-gradient iterations in the 1/c^2 inner
product on (I - S_h) v = b from v = 0 (b = W_h(0, f), every application of the
WaveHoltz operator, the FP64 Krylov vector work), inputs resident in HBM.

Prints one JSON line: grid-point updates per second over the timed steps
(value), the roofline of the time-stepping kernel (algorithmic bytes per
launch over its event-timed average duration against 8 TB/s HBM, and against
the copy rate of the library's own streaming kernel measured in the same
run), the CPU oracle's rate on a bounded sample of the same grid, and, as
extra keys, the time to residual 1e-8 of the 2048^2 FP64 configuration
(--no-square skips it).

Other modes (used to produce the committed rocprofv3 summaries):
  --workload square
                  the 2048^2 unit square, 4th-order stencil, smooth random
                  c^2 in [0.5, 2], omega = 200, 4 Gaussian sources, solved to
                  ||b - A v|| <= 1e-8 ||b|| (FP64 CG by default; --solver
                  gmres for restarted GMRES(--restart), which stagnates near
                  4e-8 on this workload); one step = one whole solve
  --mode kernel   only W_h applications (A v) of the workload, no solver;
                  with --workload cube: the 512^3 cube (c = 1 with a c = 1.5
                  ball, omega = 80, point-like source, 2nd order, FP32 state)
  --mode solve --workload cube --iters 0
                  the same cube solved towards the residual target by CG in
                  the 1/c^2 inner product with FP64 state, at most --maxit
                  iterations (default 2000 here: about 2.6 minutes at 79 ms
                  per iteration; the solve stays near 5e-5 for thousands of
                  iterations, so the target is not reached within one run);
                  prints progress every 200 iterations and one JSON line
  --mode stream   the library's streaming kernel (copy, read, write of 1 GiB)
  --mode spectrum why the cube's CG solve is long: closed-form extreme
                  eigenvalues of A for the constant-c cube, FP64 CG at 256^3
                  (omega = 40) to the target and at 512^3 for --maxit
                  iterations with Ritz estimates and true/recursive residuals
  --mode copy     a plain device copy of known size (HBM counter calibration)
  --mode batch    64 independent 2-D solves (grids 256^2, 512^2, 1024^2,
                  omega ~ U[20, 150], c = 1, 2nd order, Gaussian sources)
                  by the batched CG, against solving them one at a time
  --mode mixed    the default workload solved to the residual target in FP64
                  and by residual correction (FP64 residuals, FP32-state CG
                  corrections to 1e-3), with the FP32 and FP64 kernel rates
  --mode implicit implicit stepping (N_ITS steps per period, multigrid-
                  preconditioned CG per step) against explicit stepping:
                  time per W_h application on the random-c^2 square at 256^2
                  .. 2048^2 (omega scaled with n), and a CG solve to 1e-8 on
                  512^2 (omega = 50) with each
  --mode adjoint  receiver-misfit gradient on 1024^2 (omega = 60, 8 sources,
                  128 receivers on a ring, data from a slower inclusion):
                  forward solve, adjoint solve and checkpointed reverse sweep
                  per source, against the plain forward solves
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves before timing")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="state precision (default: fp32 on the cube except for --iters 0, fp64 otherwise)")
    ap.add_argument("--workload", choices=["square", "cube"], default="cube",
                    help="cube: 512^3 inclusion (default; --mode solve or kernel); square: 2048^2 random c^2")
    ap.add_argument("--order", type=int, choices=[2, 4], default=0, help="stencil order (default: 4 square, 2 cube)")
    ap.add_argument("--n", type=int, default=0, help="cells per axis (default: 2048 square, 512 cube)")
    ap.add_argument("--solver", choices=["cg", "gmres"], default="cg")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--ref-rtol", dest="ref_rtol", type=float, default=1e-13,
                    help="--mode mixed: tolerance of the FP64 reference solve")
    ap.add_argument("--maxit", type=int, default=0,
                    help="iteration cap of a solve to the residual target (0: 40000 square, 2000 cube)")
    ap.add_argument("--iters", type=int, default=100,
                    help="cube: Krylov iterations per timed step, CG or --solver gmres "
                         "(0: one solve towards the residual target)")
    ap.add_argument("--no-square", dest="square", action="store_false", default=True,
                    help="cube: skip the 2048^2 FP64 time-to-residual solve reported beside the line")
    ap.add_argument("--kernel", default="auto",
                    help="time-stepping kernel family (auto, node, blocked_2d, zcol_3d, blocked_3d)")
    ap.add_argument("--kblock", type=int, default=0, help="leapfrog steps per launch (0 = automatic)")
    ap.add_argument("--tile", type=int, default=0, help="tile parameter of the kernel family (0 = default)")
    ap.add_argument("--autotune", action="store_true", help="let the library time every variant first")
    ap.add_argument("--mode", choices=["solve", "kernel", "copy", "stream", "batch", "adjoint", "implicit", "mixed",
                                       "spectrum"],
                    default="solve")
    ap.add_argument("--nits", type=int, default=10, help="--mode implicit: implicit steps per period")
    ap.add_argument("--sizes", default="256,512,1024,2048", help="--mode implicit: grid sizes compared")
    ap.add_argument("--skip-solve", action="store_true", help="--mode implicit: only the per-application times")
    ap.add_argument("--fixed-sizes", default="512,1024,2048,4096",
                    help="--mode implicit: grid sizes of the fixed-omega (omega = 50) series")
    ap.add_argument("--count", type=int, default=64, help="problems in --mode batch")
    ap.add_argument("--no-sequential", dest="sequential", action="store_false", default=True,
                    help="--mode batch: skip the one-at-a-time comparison")
    ap.add_argument("--applies", type=int, default=20, help="applications timed in --mode kernel")
    ap.add_argument("--cpu-baseline", dest="cpu_baseline", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    args = ap.parse_args()
    # the cube is the workload of --mode solve and --mode kernel; the other
    # modes have workloads of their own (sizes default as for the square)
    if args.mode not in ("solve", "kernel"):
        args.workload = "square"
    cube = args.workload == "cube"
    if args.precision is None:
        block = args.mode == "solve" and args.iters > 0
        args.precision = "fp32" if cube and (args.mode == "kernel" or block) else "fp64"
    if not args.maxit:
        args.maxit = 2000 if cube else (6000 if args.mode == "spectrum" else 40000)
    if not args.order:
        args.order = 2 if cube else 4
    if not args.n:
        args.n = 512 if cube else 2048
    return args


def run_mixed(args, dev):
    """FP64 CG against mixed-precision residual correction on the default
    workload, both to the residual target."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    w = wl.smooth_random_speed_sources(n=args.n, order=4)
    solvers = {}
    for prec in ("fp64", "fp32"):
        s = Solver(2, (args.n, args.n), order=4, precision=prec, restart=2)
        s.set_c2(w["c2"])
        s.set_source(w["f"])
        s.set_frequency(w["omega"])
        solvers[prec] = s
    rates = {}
    for prec, s in solvers.items():
        v = torch.zeros(s.shape, dtype=torch.float64, device=dev)
        out = s.new()
        s.apply_A(v, out=out)
        s.profile_enable(True)
        for _ in range(10):
            s.apply_A(v, out=out)
        pr = s.profile_read()
        s.profile_enable(False)
        rates[prec] = round(pr["point_steps"] / pr["ms"] * 1e-6, 1)
    hi, lo = solvers["fp64"], solvers["fp32"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x64, i64 = hi.solve(method="cg", rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    log(f"FP64 CG: {i64['iters']} iterations, {t64:.2f}s")
    t0 = time.perf_counter()
    xm, im = hi.solve_mixed(lo, rtol=args.rtol, maxit=50, inner_method="cg", inner_rtol=1e-3, inner_maxit=5000)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    log(f"mixed: {im['iters']} corrections, {im['applies']} applies, {tm:.2f}s")
    # calibration: an FP64 solve tight enough that kappa_hat * rtol is far
    # below 1e-5 (kappa_hat from the extreme Ritz values of that solve), the
    # reference against which each solve's error is reported
    t0 = time.perf_counter()
    xr, ir = hi.solve(method="cg", rtol=args.ref_rtol, maxit=4 * args.maxit)
    torch.cuda.synchronize()
    tr = time.perf_counter() - t0
    kappa = ir["ritz_max"] / ir["ritz_min"]
    log(f"FP64 reference CG to {args.ref_rtol:g}: {ir['iters']} iterations, {tr:.2f}s, kappa_hat {kappa:.3e}")

    def err(x):
        return float(torch.linalg.vector_norm(x - xr) / torch.linalg.vector_norm(xr))

    diff = float(torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64))
    print(json.dumps({"mode": "mixed", "workload": f"square {args.n}^2, order 4, random c^2 in [0.5,2], omega=200",
                      "kernel_GPts_per_s": rates,
                      "fp64_cg": {"seconds": round(t64, 3), "iters": i64["iters"], "applies": i64["applies"],
                                  "rel_res": i64["rel_res"], "converged": i64["converged"],
                                  "helmholtz_rel_res": hi.helmholtz_residual(x64), "rel_err_to_reference": err(x64)},
                      "mixed": {"seconds": round(tm, 3), "corrections": im["iters"], "applies": im["applies"],
                                "rel_res": im["rel_res"], "converged": im["converged"],
                                "helmholtz_rel_res": hi.helmholtz_residual(xm), "rel_diff_to_fp64": diff,
                                "rel_err_to_reference": err(xm)},
                      "fp64_reference": {"rtol": args.ref_rtol, "seconds": round(tr, 3), "iters": ir["iters"],
                                         "rel_res": ir["rel_res"], "converged": ir["converged"],
                                         "ritz_min": ir["ritz_min"], "ritz_max": ir["ritz_max"],
                                         "kappa_hat": kappa, "kappa_hat_times_rtol": kappa * args.ref_rtol,
                                         "kappa_hat_times_target": kappa * args.rtol}}),
          flush=True)


def run_implicit(args, dev):
    """Implicit against explicit stepping on the random-c^2 square (4th order,
    FP64): per-application times at fixed points per wavelength and one solve
    to the residual target."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    rows = []
    for n in [int(x) for x in args.sizes.split(",")]:
        omega = 200.0 * n / 2048
        w = wl.smooth_random_speed_sources(n=n, order=4, omega=omega)
        s = Solver(2, (n, n), order=4, restart=2)
        s.set_c2(w["c2"])
        s.set_source(w["f"])
        tp_e = s.set_frequency(omega)
        g = torch.Generator(device=dev)
        g.manual_seed(7)
        v = torch.randn(s.shape, dtype=torch.float64, device=dev, generator=g)
        out = s.new()

        def per_apply(reps):
            s.apply_A(v, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s.apply_A(v, out=out)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        te = per_apply(10)
        s.set_implicit(args.nits, 1e-10)
        s.set_frequency(omega)
        st0 = s.implicit_stats()
        ti = per_apply(3)
        st1 = s.implicit_stats()
        inner = (st1["inner_iters"] - st0["inner_iters"]) / max(1, st1["steps"] - st0["steps"])
        rows.append({"n": n, "omega": omega, "explicit_nt": tp_e["nt"], "explicit_ms_per_apply": round(te * 1e3, 3),
                     "implicit_nits": args.nits, "implicit_ms_per_apply": round(ti * 1e3, 3),
                     "inner_cg_iters_per_step": round(inner, 2), "mg_levels": st1["levels"],
                     "implicit_ns_per_node_step": round(ti * 1e9 / ((n - 1) ** 2 * args.nits), 3)})
        log(f"implicit vs explicit: {rows[-1]}")
        del s
        torch.cuda.empty_cache()
    # fixed omega: the explicit N_t grows like n, the implicit one does not
    fixed = []
    for n in ([] if args.skip_solve else [int(x) for x in args.fixed_sizes.split(",") if x]):
        omega = 50.0
        w = wl.smooth_random_speed_sources(n=n, order=4, omega=omega)
        s = Solver(2, (n, n), order=4, restart=2)
        s.set_c2(w["c2"])
        s.set_source(w["f"])
        tp_e = s.set_frequency(omega)
        del w
        g = torch.Generator(device=dev)
        g.manual_seed(8)
        v = torch.randn(s.shape, dtype=torch.float64, device=dev, generator=g)  # a zero input skips the solves
        out = s.new()

        def per_apply_fixed(reps):
            s.apply_A(v, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s.apply_A(v, out=out)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        te = per_apply_fixed(3)
        s.set_implicit(args.nits, 1e-10)
        s.set_frequency(omega)
        ti = per_apply_fixed(2)
        fixed.append({"n": n, "omega": omega, "explicit_nt": tp_e["nt"], "explicit_ms_per_apply": round(te * 1e3, 3),
                      "implicit_nits": args.nits, "implicit_ms_per_apply": round(ti * 1e3, 3)})
        log(f"fixed omega: {fixed[-1]}")
        del s
        torch.cuda.empty_cache()
    n, omega = 512, 50.0
    w = wl.smooth_random_speed_sources(n=n, order=4, omega=omega)
    solves = {}
    for mode in (() if args.skip_solve else ("explicit", "implicit")):
        s = Solver(2, (n, n), order=4, restart=2)
        s.set_c2(w["c2"])
        s.set_source(w["f"])
        if mode == "implicit":
            s.set_implicit(args.nits, 1e-10)
        s.set_frequency(omega)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(method="cg", rtol=args.rtol, maxit=20000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves[mode] = {"seconds": round(dt, 3), "iters": info["iters"], "applies": info["applies"],
                        "converged": info["converged"], "rel_res": info["rel_res"],
                        "helmholtz_rel_res": s.helmholtz_residual(x)}
        log(f"solve 512^2 {mode}: {solves[mode]}")
        del s
    print(json.dumps({"mode": "implicit", "workload": "square, order 4, random c^2 in [0.5,2], omega = 200 n/2048, "
                      "4 Gaussian sources, FP64; implicit steps solved by CG with a multigrid V-cycle to 1e-10",
                      "per_apply": rows, "per_apply_fixed_omega_50": fixed, "solve_512": solves}), flush=True)


def run_cube_kernel(args, dev):
    """The 512^3 cube (c = 1 with a c = 1.5 ball, omega = 80, point-like
    source): A v applications only, timed with events on the library's
    stream."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    n = args.n
    w = wl.cube_inclusion(n=n, order=args.order)
    s = Solver(3, (n, n, n), order=args.order, precision=args.precision)
    s.set_tuning(args.kernel, args.kblock, args.tile)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    del w
    tun = s.tuning()
    log(f"cube {n}^3 p={args.order} {args.precision}: time params {tp}, tuning {tun}")
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    v = torch.randn(s.shape, dtype=torch.float64, device=dev, generator=g)
    out = s.new()
    for _ in range(2):
        s.apply_A(v, out=out)
    torch.cuda.synchronize()
    s.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.applies):
        s.apply_A(v, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pr = s.profile_read()
    s.profile_enable(False)
    print(json.dumps({"mode": "kernel", "workload": f"cube {n}^3, order {args.order}, c = 1 with a c = 1.5 ball, "
                      f"omega = {tp['omega']}", "precision": args.precision, "kernel": tun["kernel"],
                      "kblock": tun["kblock"], "tile": tun["tile"], "nt": tp["nt"], "applies": args.applies,
                      "ms_per_apply": dt / args.applies * 1e3, "launches": pr["launches"],
                      "us_per_launch": pr["ms"] / pr["launches"] * 1e3,
                      "alg_GBps": pr["bytes"] / pr["ms"] * 1e-6,
                      "GPts_per_s": pr["point_steps"] / pr["ms"] * 1e-6}), flush=True)


def run_cube_solve(args, dev):
    """The 512^3 cube (omega = 80) solved once from v = 0 to the residual
    target by CG in the 1/c^2 inner product; the time to residual is taken
    from the solve call with the inputs resident and the context set up."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    n = args.n
    w = wl.cube_inclusion(n=n, order=args.order)
    s = Solver(3, (n, n, n), order=args.order, precision=args.precision, restart=2)
    s.set_tuning(args.kernel, args.kblock, args.tile)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    del w
    tun = s.tuning()
    log(f"cube {n}^3 p={args.order} {args.precision}: time params {tp}, tuning {tun}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def progress(k, rel):
        if k % 200 == 0:
            log(f"  iteration {k}: relative residual {rel:.3e} after {time.perf_counter() - t0:.1f}s")

    x, info = s.solve(method="cg", rtol=args.rtol, maxit=args.maxit, callback=progress)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    unknowns = (n - 1) ** 3
    print(json.dumps({"mode": "solve", "workload": f"cube {n}^3, order {args.order}, c = 1 with a c = 1.5 ball, "
                      f"omega = {tp['omega']}, point-like source, CG (1/c^2 inner product)",
                      "precision": args.precision, "kernel": tun["kernel"], "kblock": tun["kblock"],
                      "tile": tun["tile"], "nt": tp["nt"], "rtol": args.rtol, "converged": bool(info["converged"]),
                      "iterations": info["iters"], "applies": info["applies"], "rel_res": info["rel_res"],
                      "helmholtz_rel_res": s.helmholtz_residual(x), "time_to_residual_s": t,
                      "GPts_per_s": unknowns * tp["nt"] * info["applies"] / t * 1e-9}), flush=True)


def unblocked_bytes(precision, cvar, forcing):
    """Algorithmic bytes of one point-step taken one step per pass: W^n and
    W^{n-1} read, W^{n+1} written (state precision), c^2 and f read when
    present, the FP64 accumulator read and written."""
    t = 8 if precision == "fp64" else 4
    return 3 * t + (t if cvar else 0) + (t if forcing else 0) + 16


def cpu_baseline_grid(dim, n, order, c2, omega, steps, threads=None):
    """The FP64 CPU oracle on a bounded sample of a workload: W_h(v, 0) with
    `steps` leapfrog steps per period on the full grid, c^2 and frequency of
    the workload (the time-step size of the full period; only the step count
    is cut).  Returns GPts/s, the thread count and the seconds."""
    from oracle import core as oc
    import workloads as wl
    grid = oc.Grid(dim, (n,) * dim, order)
    tp = dict(oc.time_params(grid, c2, omega), nt=int(steps), periods=1)
    v = wl.random_field(grid.shape, seed=99)
    prev = oc.max_threads()
    if threads:
        oc.set_threads(threads)
    try:
        used = oc.max_threads()
        t0 = time.perf_counter()
        oc.apply(grid, c2, None, v, tp, with_forcing=False)
        sec = time.perf_counter() - t0
    finally:
        oc.set_threads(prev)
    return grid.unknowns * tp["nt"] / sec / 1e9, used, sec


def run_c1(dev, reps=5):
    """The 128^2 single-Gaussian configuration end to end on the GPU: 30
    fixed-point iterations from v = 0 (FP64, 2nd order, c = 1, omega = 10.3),
    the best of `reps` timed runs after one untimed; returns the record and
    the workload (for the CPU oracle's run of the same iterations)."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    w = wl.single_gaussian_source()
    s = Solver(2, (w["n"], w["n"]), order=2, precision="fp64", restart=2)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    s.solve(method="fpi", rtol=0.0, maxit=w["fpi_iters"])
    best, info = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(method="fpi", rtol=0.0, maxit=w["fpi_iters"])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        best = t if best is None else min(best, t)
    pts = (w["n"] - 1) ** 2 * tp["nt"] * info["applies"]
    return {"workload": "square 128^2, order 2, c = 1, omega = 10.3, Gaussian exp(-200|x-(0.4,0.6)|^2), "
                        "30 fixed-point iterations, FP64",
            "seconds": round(best, 5), "applies": info["applies"], "nt": tp["nt"],
            "GPts_per_s": round(pts / best * 1e-9, 3), "cr_last": info["cr_last"],
            "mu_pred": info["mu_pred"]}, w


def cpu_c1(w):
    """The FP64 CPU oracle's 30 fixed-point iterations of the 128^2
    configuration, end to end."""
    from oracle import core as oc
    grid = oc.Grid(2, (w["n"], w["n"]), 2)
    tp = oc.time_params(grid, w["c2"], w["omega"])
    t0 = time.perf_counter()
    oc.fpi(grid, w["c2"], w["f"], tp, w["fpi_iters"])
    return time.perf_counter() - t0


def run_square_reference(dev, log_every=0):
    """One FP64 CG solve of the 2048^2 configuration to the residual target
    (after one untimed application): time to residual and rate."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    w = wl.smooth_random_speed_sources(n=2048, order=4)
    s = Solver(2, (2048, 2048), order=4, precision="fp64", restart=2)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    s.apply_A(s.new(), out=s.new())
    torch.cuda.synchronize()
    s.profile_enable(True)
    t0 = time.perf_counter()
    x, info = s.solve(method="cg", rtol=1e-8, maxit=40000)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile_enable(False)
    launch_us = prof["ms"] / prof["launches"] * 1e3
    achieved = prof["bytes"] / prof["launches"] / (launch_us * 1e-6) / 1e9
    out = {"workload": "square 2048^2, order 4, random c^2 in [0.5,2], omega=200, 4 Gaussian sources, FP64, "
                       "CG (1/c^2 inner product) to 1e-8",
           "time_to_residual_s": round(t, 3), "converged": bool(info["converged"]), "iterations": info["iters"],
           "applies": info["applies"], "rel_res": info["rel_res"], "helmholtz_rel_res": s.helmholtz_residual(x),
           "GPts_per_s": round(2047 ** 2 * tp["nt"] * info["applies"] / t * 1e-9, 2),
           # the stepping kernel over the whole solve (HIP events on the library's stream)
           "kernel": {"name": "block_steps_kernel", "steps_per_launch": s.tuning()["kblock"],
                      "launch_us": round(launch_us, 3), "bytes_per_launch": prof["bytes"] / prof["launches"],
                      "achieved_GBps": round(achieved, 1), "frac_of_8TBps": round(achieved / 8000.0, 4),
                      "stepping_share": round(prof["ms"] * 1e-3 / t, 4)}}
    del s, x
    torch.cuda.empty_cache()
    return out


def run_cube_block(args, dev):
    """The default benchmark: fixed blocks of CG iterations on the 512^3
    inclusion cube with FP32 state and FP64 filter and Krylov vectors."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    n, order = args.n, args.order
    t_setup = time.perf_counter()
    w = wl.cube_inclusion(n=n, order=order)
    gmres = args.solver == "gmres"
    s = Solver(3, (n, n, n), order=order, precision=args.precision, restart=args.restart if gmres else 2)
    s.set_tuning(args.kernel, args.kblock, args.tile)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    tun = s.tuning()
    log(f"cube {n}^3 p={order} {args.precision}: set up in {time.perf_counter() - t_setup:.1f}s, "
        f"time params {tp}, tuning {tun}")
    unknowns = (n - 1) ** 3
    pts_per_apply = unknowns * tp["nt"] * tp["periods"]

    def one_step():
        return s.solve(method=args.solver, rtol=0.0, maxit=args.iters,
                       restart=args.restart if gmres else 2)

    for i in range(args.warmup):
        t0 = time.perf_counter()
        one_step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup}: {time.perf_counter() - t0:.2f}s")
    s.profile_enable(True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x, info = one_step()
        infos.append(info)
        log(f"step {i + 1}/{args.steps}: {info['iters']} {args.solver} iterations, {info['applies']} applies, "
            f"rel_res {info['rel_res']:.3e}, {info['seconds']:.2f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile_enable(False)
    helm = s.helmholtz_residual(x)
    del x
    applies = sum(i["applies"] for i in infos)
    value = applies * pts_per_apply / elapsed / 1e9
    launch_us = prof["ms"] / prof["launches"] * 1e3
    bytes_per_launch = prof["bytes"] / prof["launches"]
    achieved = bytes_per_launch / (launch_us * 1e-6) / 1e9
    kname = {"blocked_2d": "block_steps_kernel", "blocked_3d": "block3d_steps_kernel",
             "node": "step_kernel"}.get(tun["kernel"], tun["kernel"])
    del s
    torch.cuda.empty_cache()
    ceil = stream_ceilings(dev)
    log(f"streaming kernel: {ceil}")
    ub = unblocked_bytes(args.precision, True, False)
    result = {
        "metric": "grid-pt updates/s (GPts/s, % HBM roofline) + time to Helmholtz residual 1e-8",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded random inclusion and point-like Gaussian source)",
        "config": {
            "workload": f"cube {n}^3, order {order}, c = 1 with a c = 1.5 ball, omega = {w['omega']:g}, "
                        f"point-like Gaussian source; {args.precision} state, FP64 filter and Krylov; "
                        f"step = {args.iters} "
                        + (f"GMRES({args.restart}) iterations" if gmres else "CG iterations (1/c^2 inner product)")
                        + " from v = 0",
            "n": n, "order": order, "omega": w["omega"], "nt": tp["nt"], "solver": args.solver,
            "restart": args.restart if gmres else None,
            "iterations_per_step": args.iters, "state_precision": args.precision,
            "filter_and_krylov_precision": "fp64", "kernel": tun["kernel"], "steps_per_launch": tun["kblock"],
            "tile_rows": tun["tile"], "owned_tile": list(tun["owned"]),
        },
        "time_to_residual_s": None,
        "rel_res_after_step": infos[-1]["rel_res"],
        "helmholtz_rel_res_after_step": helm,
        "applies_per_step": infos[-1]["applies"],
        "stepping_share": round(prof["ms"] * 1e-3 / elapsed, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, {"n": n, "order": order, "precision": args.precision,
                                                "kblock": tun["kblock"], "tile_rows": tun["tile"]}),
            "bytes_per_launch": bytes_per_launch,
            "launch_us": round(launch_us, 3),
            "launches": prof["launches"],
            "measured_copy_GBps": ceil["copy_GBps"],
            "frac_of_measured_copy": round(achieved / ceil["copy_GBps"], 4),
            # the same 36-byte-per-node mix streamed elementwise (no stencil,
            # no halo): the practical ceiling for this kernel's algorithmic bytes
            "measured_pass_mix_GBps": ceil["pass_mix_GBps"],
            "frac_of_measured_pass_mix": round(achieved / ceil["pass_mix_GBps"], 4),
            "stream_kernel_GBps": ceil,
            "kernel_GPts_per_s": round(prof["point_steps"] / prof["ms"] * 1e-6, 2),
            "unblocked_bytes_per_point_step": ub,
            "kernel_GPts_vs_unblocked_roofline": round(prof["point_steps"] / prof["ms"] * 1e-6 / (HBM_PEAK_GBS / ub),
                                                       3),
        },
    }
    if args.square:
        log("2048^2 FP64 CG solve to 1e-8 (time to residual)")
        result["square_fp64_time_to_residual"] = run_square_reference(dev)
    log("128^2 single-Gaussian configuration: 30 fixed-point iterations")
    c1, w1 = run_c1(dev)
    result["c1_fpi_30_iterations"] = c1
    if args.cpu_baseline:
        steps = 24
        log(f"CPU oracle baseline: {steps} leapfrog steps of the {n}^3 grid on the host cores")
        rate, cores, sec = cpu_baseline_grid(3, n, order, w["c2"], w["omega"], steps)
        steps1 = 5
        rate1, _, sec1 = cpu_baseline_grid(3, n, order, w["c2"], w["omega"], steps1, threads=1)
        result["cpu_baseline"] = {
            "value": round(rate, 4), "unit": "GPts/s", "cores": cores, "kind": "oracle",
            "sample": f"W_h(v, 0) over {steps} leapfrog steps of the same {n}^3 grid, c^2 and time step "
                      f"({unknowns} unknowns), FP64, {sec:.1f}s on {cores} threads",
            "single_thread_value": round(rate1, 4),
            "single_thread_sample": f"{steps1} leapfrog steps of the same grid on one thread, {sec1:.1f}s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
        }
        sec_c1 = cpu_c1(w1)
        result["cpu_baseline"]["c1_end_to_end_s"] = round(sec_c1, 3)
        result["c1_fpi_30_iterations"]["cpu_oracle_s"] = round(sec_c1, 3)
    print(json.dumps(result), flush=True)


def run_spectrum(args, dev):
    """Why the 512^3 cube's CG solve is long: the closed-form extreme
    eigenvalues of A = I - S_h over the sine modes of the constant-c cube
    (background c = 1 and the inclusion's c = 1.5) at 256^3 (omega = 40) and
    512^3 (omega = 80), the same points per wavelength; FP64 CG on the
    inclusion cube at 256^3 to the residual target and at 512^3 for --maxit
    iterations, each with the extreme Ritz values of its Lanczos matrix
    (estimates of A's extreme eigenvalues) and the true against the recursive
    residual at exit; and the iteration count at 512^3 predicted from them."""
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver
    out = {"mode": "spectrum"}
    for n, omega, maxit in ((256, 40.0, 40000), (512, 80.0, args.maxit)):
        w = wl.cube_inclusion(n=n, order=2, omega=omega)
        s = Solver(3, (n, n, n), order=2, precision="fp64", restart=2)
        s.set_c2(w["c2"])
        s.set_source(w["f"])
        tp = s.set_frequency(w["omega"])
        del w
        rec = {"n": n, "omega": omega, "nt": tp["nt"]}
        for c2 in (1.0, 2.25):
            t0 = time.perf_counter()
            lo, hi, k = s.filter_spectrum(c2)
            rec[f"closed_form_c2_{c2:g}"] = {"a_min": lo, "a_max": hi, "kappa": hi / lo, "mode_at_min": k,
                                              "seconds": round(time.perf_counter() - t0, 2)}
            log(f"{n}^3 omega {omega}: c^2 = {c2:g}: 1 - beta_d in [{lo:.3e}, {hi:.3f}], kappa {hi / lo:.3e}, "
                f"closest mode {k}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []

        def progress(kk, rel):
            if kk % 500 == 0:
                hist.append((kk, rel))
                log(f"  {n}^3 iteration {kk}: relative residual {rel:.3e} after {time.perf_counter() - t0:.1f}s")

        x, info = s.solve(method="cg", rtol=args.rtol, maxit=maxit, callback=progress)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rec["cg"] = {"iterations": info["iters"], "converged": bool(info["converged"]), "seconds": round(t, 2),
                     "ms_per_iteration": round(t / max(info["iters"], 1) * 1e3, 2),
                     "rel_res_true": info["rel_res"], "rel_res_recursive": info["rel_res_recursive"],
                     "ritz_min": info["ritz_min"], "ritz_max": info["ritz_max"],
                     "kappa_ritz": info["ritz_max"] / info["ritz_min"], "history": hist[-40:],
                     "helmholtz_rel_res": s.helmholtz_residual(x)}
        log(f"{n}^3: {info['iters']} iterations, true {info['rel_res']:.3e}, recursive "
            f"{info['rel_res_recursive']:.3e}, Ritz [{info['ritz_min']:.3e}, {info['ritz_max']:.3f}]")
        out[f"cube{n}"] = rec
        del s, x
        torch.cuda.empty_cache()
    # CG needs about sqrt(kappa)/2 ln(2/eps) iterations; scale the iteration
    # count measured at 256^3 by the ratio of the two Ritz estimates
    a, b = out["cube256"]["cg"], out["cube512"]["cg"]
    if a["converged"]:
        pred = a["iterations"] * math.sqrt(b["kappa_ritz"] / a["kappa_ritz"])
        out["predicted_iterations_512"] = round(pred)
        out["predicted_time_to_residual_512_s_extrapolated"] = round(pred * b["ms_per_iteration"] * 1e-3, 1)
    out["bound_iterations_512"] = round(0.5 * math.sqrt(b["kappa_ritz"]) * math.log(2.0 / args.rtol))
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CSRC = os.path.join(ROOT, "paper_2504_03074_amd", "csrc")
# committed rocprofv3 HBM-counter summaries: (summary file, kernel source it was taken from)
COUNTER_SUMMARIES = {
    "block_steps_kernel": (os.path.join(ROOT, "profiles", "block_steps_kernel_square2048_p4_fp64_hbm_counters.txt"),
                           os.path.join(CSRC, "wh_block_impl.h")),
    "block3d_steps_kernel": (os.path.join(ROOT, "profiles", "block3d_steps_kernel_cube512_p2_fp32_hbm_counters.txt"),
                             os.path.join(CSRC, "wh_block3d_impl.h")),
}


def measured_traffic(kernel, match):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    summary's workload fields differ from `match` or the kernel source changed
    since the counters were taken."""
    import hashlib
    if kernel not in COUNTER_SUMMARIES:
        return None
    summary, source = COUNTER_SUMMARIES[kernel]
    if not os.path.exists(summary):
        return None
    fields = {}
    for line in open(summary):
        if "=" in line:
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    if any(fields.get(k) != str(v) for k, v in match.items()):
        return None
    return float(fields["traffic_bytes_per_launch"])


def stream_ceilings(dev, nbytes=1 << 30):
    """GB/s of the library's streaming kernel: copy, read and write of
    `nbytes`, each the average of 10 launches after one untimed."""
    import torch
    from paper_2504_03074_amd.wh import wh_stream_bandwidth
    a = torch.zeros(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes), (2, "write", nbytes)):
        ms = wh_stream_bandwidth(kind, a.data_ptr(), b.data_ptr(), nbytes, 0, 10, stream)
        out[f"{name}_GBps"] = round(moved / (ms * 1e-3) * 1e-9, 1)
    del a, b
    # the FP32 blocked pass's per-node traffic (three FP32 arrays and the FP64
    # accumulator read, two FP32 arrays and the accumulator written: 36 B) on
    # 2^27 nodes, elementwise with 16-byte accesses: the ceiling for that mix
    nodes = 1 << 27
    src = torch.zeros(nodes * 3, dtype=torch.float32, device=dev)
    dst = torch.zeros(nodes * 4, dtype=torch.float32, device=dev)
    ms = wh_stream_bandwidth(3, src.data_ptr(), dst.data_ptr(), 36 * nodes, 0, 10, stream)
    out["pass_mix_GBps"] = round(36 * nodes / (ms * 1e-3) * 1e-9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, order, nt_sample):
    """The FP64 CPU oracle on a bounded sample of the workload: one W_h(v, 0)
    application of the same grid, c^2 and frequency (all its leapfrog steps),
    on the host cores.  Returns GPts/s, the thread count and the seconds."""
    import numpy as np
    from oracle import core as oc
    import workloads as wl
    grid = oc.Grid(2, (w["n"], w["n"]), order)
    tp = oc.time_params(grid, w["c2"], w["omega"])
    if nt_sample:
        tp = dict(tp, nt=int(nt_sample))
    v = wl.random_field(grid.shape, seed=99)
    t0 = time.perf_counter()
    oc.apply(grid, w["c2"], None, v, tp, with_forcing=False)
    sec = time.perf_counter() - t0
    pts = grid.unknowns * tp["nt"] * tp["periods"]
    return pts / sec / 1e9, oc.max_threads(), sec, tp["nt"]


def cpu_single_thread(w, order, steps=12):
    """The same oracle on one thread, over `steps` leapfrog steps of the same
    grid (the rate per point-step does not depend on the step count)."""
    from oracle import core as oc
    threads = oc.max_threads()
    oc.set_threads(1)
    try:
        rate, _, sec, nt = cpu_baseline(w, order, steps)
    finally:
        oc.set_threads(threads)
    return rate, sec, nt


def cpu_model():
    """Model name of the host CPU with its family/model/stepping numbers (a
    virtualised host may report only a short name) and the logical CPU count."""
    name, fam, mod, step, logical = "unknown", "?", "?", "?", 0
    try:
        for line in open("/proc/cpuinfo"):
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key == "processor":
                logical += 1
            elif key == "model name" and name == "unknown":
                name = val
            elif key == "cpu family" and fam == "?":
                fam = val
            elif key == "model" and mod == "?":
                mod = val
            elif key == "stepping" and step == "?":
                step = val
    except OSError:
        pass
    return f"{name} (family {fam}, model {mod}, stepping {step}; {logical} logical CPUs in /proc/cpuinfo)"


def run_batch(args, dev):
    """Many independent solves at once: the batched CG (one launch per blocked
    pass over all problems, the iteration replayed from a HIP graph) against
    the same solves one at a time through the single-problem path."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Batch, Solver

    probs = wl.batched_problems(args.count)
    solvers = []
    for p in probs:
        s = Solver(2, (p["n"], p["n"]), order=p["order"], precision=args.precision, restart=2)
        s.set_c2(p["c2"])
        s.set_source(wl.materialise_source(2, p["n"], p["source"]))
        s.set_frequency(p["omega"], periods=p["periods"], cfl_frac=p["cfl"])
        solvers.append(s)
    batch = Batch(solvers, kblock=args.kblock, tile=args.tile)
    if args.autotune:
        log(f"batch autotune: {batch.autotune(3)}")
    tun = batch.tuning()
    nts = [s.time_params["nt"] for s in solvers]
    pts_apply = [(p["n"] - 1) ** 2 * nt for p, nt in zip(probs, nts)]
    log(f"{len(probs)} problems, nt {min(nts)}..{max(nts)}, sizes "
        + ", ".join(f"{n}^2 x{sum(p['n'] == n for p in probs)}" for n in (256, 512, 1024)))

    # batched apply: algorithmic bytes over event-timed duration
    zeros = [s.new() for s in solvers]
    outs = [s.new() for s in solvers]
    batch.apply(zeros, with_forcing=False, outs=outs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(args.applies // 4, 3)
    e0.record()
    for _ in range(reps):
        batch.apply(zeros, with_forcing=False, outs=outs)
    e1.record()
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / reps
    T = 8 if args.precision == "fp64" else 4
    kb = tun["kblock"]
    alg_bytes = 0.0
    for p, nt in zip(probs, nts):
        interior = (p["n"] - 1) ** 2
        passes = math.ceil((nt * p["periods"] - 1) / kb)
        # first step: v read, W^0, W^1 and the accumulator written; each
        # pass: two levels read and written, accumulator read and written
        alg_bytes += interior * ((8 + 2 * T + 8) + passes * (4 * T + 16))
    achieved = alg_bytes / (apply_ms * 1e-3) / 1e9

    def progress(k, rel):
        if k % 500 == 0:
            log(f"  iteration {k}: worst residual estimate {rel:.3e}")

    for i in range(args.warmup):
        log(f"warmup batched solve {i + 1}/{args.warmup}")
        batch.solve(rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        xs, infos = batch.solve(rtol=args.rtol, maxit=args.maxit, callback=progress)
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    pts = sum(i["applies"] * pa for i, pa in zip(infos, pts_apply))
    value = pts / elapsed / 1e9
    its = [i["iters"] for i in infos]
    helms = [s.helmholtz_residual(x) for s, x in zip(solvers, xs)]
    helm = max(helms)
    worst = int(np.argmax(helms))
    log(f"batched: {elapsed:.2f}s, {value:.1f} GPts/s, iterations {min(its)}..{max(its)}")

    seq = None
    if args.sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        spts = 0
        for s, pa in zip(solvers, pts_apply):
            x, inf = s.solve(method="cg", rtol=args.rtol, maxit=args.maxit)
            spts += inf["applies"] * pa
        torch.cuda.synchronize()
        st = time.perf_counter() - t0
        seq = {"time_to_residual_s": round(st, 4), "GPts_per_s": round(spts / st / 1e9, 3)}
        log(f"one at a time: {st:.2f}s, {spts / st / 1e9:.1f} GPts/s")

    result = {
        "metric": "grid-pt updates/s (GPts/s, % HBM roofline) + time to Helmholtz residual 1e-8",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-state/f64-acc",
        "data": "synthetic (seeded frequencies, sizes and Gaussian sources)",
        "config": {
            "workload": f"{len(probs)} batched 2-D solves, grids {{256,512,1024}}^2, omega ~ U[20,150], c = 1, "
                        f"2nd order, one Gaussian source each, batched CG to {args.rtol:g}",
            "problems": len(probs), "rtol": args.rtol, "precision": args.precision,
            "steps_per_launch": kb, "tile_rows": tun["tile"], "autotuned": bool(args.autotune),
        },
        "time_to_residual_s": round(elapsed, 4),
        "converged": all(i["converged"] for i in infos),
        "max_rel_res": max(i["rel_res"] for i in infos),
        "helmholtz_rel_res_max": helm,
        # the Helmholtz residual weights an error mode by |omega^2 - lambda^2|
        # where the WaveHoltz residual weights it by |1 - beta_d|; near
        # resonance the ratio is large (the worst problem and why: design notes)
        "helmholtz_worst_problem": {"n": probs[worst]["n"], "omega": probs[worst]["omega"],
                                    "rel_res": infos[worst]["rel_res"], "helmholtz_rel_res": helms[worst]},
        "iters_min_median_max": [min(its), int(np.median(its)), max(its)],
        "sequential": seq,
        "speedup_vs_sequential": round(seq["time_to_residual_s"] / elapsed, 3) if seq else None,
        "roofline": {
            "bound": "hbm", "kernel": "batch_block_steps_kernel (+ batch_first_step_kernel)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_apply": alg_bytes, "apply_ms": round(apply_ms, 4),
        },
    }
    print(json.dumps(result), flush=True)


def run_adjoint(args, dev):
    """Gradient of J(c^2, f) = 1/2 sum_s ||R v*_s - d_s||^2 with respect to
    c^2 and every source: per source a forward solve, the receiver misfit,
    the adjoint solve (I - S)^T lam = R^T (R v* - d) and the checkpointed
    reverse sweep, all to the same residual as the forward solves."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver

    n = 1024 if args.n == 2048 else args.n
    w = wl.adjoint_problem(n=n)
    nsrc = len(w["sources"])
    idx = torch.from_numpy(w["receivers"]).to(dev)
    s = Solver(2, (n, n), order=w["order"], restart=2)
    s.set_c2(w["c2_true"])
    tp = s.set_frequency(w["omega"], periods=w["periods"], cfl_frac=w["cfl"])
    nt = tp["nt"]
    log(f"adjoint workload {n}^2, omega {w['omega']}, nt {nt}, {nsrc} sources, {idx.numel()} receivers")
    data = []
    for f in w["sources"]:  # observations from the true model (untimed)
        s.set_source(f)
        u, inf = s.solve(method="cg", rtol=args.rtol * 1e-2, maxit=args.maxit)
        data.append(u.reshape(-1)[idx].clone())
    s.set_c2(w["c2_background"])
    s.set_frequency(w["omega"], periods=w["periods"], nt=nt)
    sources = [torch.from_numpy(f).to(dev) for f in w["sources"]]
    unknowns = (n - 1) ** 2
    pts_apply = unknowns * nt * w["periods"]

    def forward_only():
        applies = 0
        for f in sources:
            s.set_source(f)
            _, inf = s.solve(method="cg", rtol=args.rtol, maxit=args.maxit)
            applies += inf["applies"]
        return applies

    def gradient():
        J = 0.0
        g_c2 = torch.zeros_like(sources[0])
        g_f = []
        applies = 0
        for f, d in zip(sources, data):
            s.set_source(f)
            v, inf = s.solve(method="cg", rtol=args.rtol, maxit=args.maxit)
            Js, gv = s.receiver_misfit(v, idx, d)
            lam, ainf = s.solve_adjoint(gv, method="cg", rtol=args.rtol, maxit=args.maxit)
            gr = s.gradient(v, lam, c2=True, f=True)
            g_c2 += gr["c2"]
            g_f.append(gr["f"])
            J += Js
            applies += inf["applies"] + ainf["applies"]
        return J, g_c2, g_f, applies

    for i in range(args.warmup):
        log(f"warmup gradient {i + 1}/{args.warmup}")
        gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        J, g_c2, g_f, applies = gradient()
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    # one reverse sweep per source: a forward sweep for the checkpoints, the
    # recomputed segments (about one more) and the reverse steps
    sweep_pts = nsrc * 3 * pts_apply
    value = (applies * pts_apply + sweep_pts) / elapsed / 1e9
    log(f"gradient: J = {J:.6e}, {elapsed:.2f}s, {applies} applies")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fapplies = forward_only()
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    log(f"forward solves only: {tf:.2f}s, {fapplies} applies")
    gm = g_c2.reshape(n + 1, n + 1)
    peak = np.unravel_index(int(torch.argmax(gm.abs()).item()), gm.shape)
    result = {
        "metric": "grid-pt updates/s (GPts/s, % HBM roofline) + time to Helmholtz residual 1e-8",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded sources and inclusion; observations from the true model)",
        "config": {
            "workload": f"receiver-misfit gradient, {n}^2, 2nd order, omega={w['omega']}, {nsrc} Gaussian sources, "
                        f"{idx.numel()} ring receivers, CG forward and adjoint solves to {args.rtol:g}",
            "n": n, "nt": nt, "sources": nsrc, "receivers": int(idx.numel()), "rtol": args.rtol,
        },
        "time_to_gradient_s": round(elapsed, 4),
        "forward_solves_s": round(tf, 4),
        "gradient_over_forward": round(elapsed / tf, 3),
        "misfit": J,
        "grad_c2_norm": float(g_c2.norm()),
        "grad_c2_peak_at": [int(peak[1]) / n, int(peak[0]) / n],
        "inclusion_centre": list(w["bump_centre"]),
        "applies": applies,
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the WaveHoltz library runs on one GPU only; multi-GPU sharding is designed "
                                   "(slab decomposition with halo exchange) but not built",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl
    from paper_2504_03074_amd import Solver

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU: the WaveHoltz path has no CPU fallback")
    dev = torch.device("cuda", 0)

    if args.mode == "copy":
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).normal_()
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 10
        for _ in range(reps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        print(json.dumps({"mode": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "GBps": 2 * nbytes / dt / 1e9}), flush=True)
        return

    if args.mode == "batch":
        run_batch(args, dev)
        return
    if args.mode == "adjoint":
        run_adjoint(args, dev)
        return
    if args.mode == "implicit":
        run_implicit(args, dev)
        return
    if args.mode == "mixed":
        run_mixed(args, dev)
        return
    if args.mode == "stream":
        print(json.dumps({"mode": "stream", "bytes": 1 << 30, **stream_ceilings(dev)}), flush=True)
        return
    if args.mode == "spectrum":
        run_spectrum(args, dev)
        return
    if args.workload == "cube":
        if args.mode == "kernel":
            run_cube_kernel(args, dev)
        elif args.iters > 0:
            run_cube_block(args, dev)
        else:
            run_cube_solve(args, dev)
        return

    order = args.order
    t_setup = time.perf_counter()
    w = wl.smooth_random_speed_sources(n=args.n, order=order)
    log(f"inputs generated in {time.perf_counter() - t_setup:.1f}s")
    s = Solver(2, (args.n, args.n), order=order, precision=args.precision,
               restart=args.restart if args.solver == "gmres" else 2)
    s.set_tuning(args.kernel, args.kblock, args.tile)
    s.set_c2(w["c2"])
    s.set_source(w["f"])
    tp = s.set_frequency(w["omega"])
    if args.autotune:
        log(f"autotune: {s.autotune(3)}")
    tun = s.tuning()
    kblock = tun["kblock"]
    tile_x, tile_y = tun["owned"]
    log(f"time params {tp}, tuning {tun}")
    unknowns = (args.n - 1) ** 2
    pts_per_apply = unknowns * tp["nt"] * tp["periods"]

    if args.mode == "kernel":
        v = torch.from_numpy(wl.random_field(s.shape, seed=5)).to(dev)
        out = s.new()
        for _ in range(2):
            s.apply_A(v, out=out)
        torch.cuda.synchronize()
        s.profile_enable(True)
        t0 = time.perf_counter()
        for i in range(args.applies):
            s.apply_A(v, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pr = s.profile_read()
        s.profile_enable(False)
        print(json.dumps({"mode": "kernel", "applies": args.applies, "ms_per_apply": dt / args.applies * 1e3,
                          "launches": pr["launches"], "us_per_launch": pr["ms"] / pr["launches"] * 1e3,
                          "alg_GBps": pr["bytes"] / pr["ms"] * 1e-6,
                          "GPts_per_s": pr["point_steps"] / pr["ms"] * 1e-6}), flush=True)
        return

    def progress(k, rel):
        if k % 1000 == 0:
            log(f"  iteration {k}: residual estimate {rel:.3e}")

    def one_solve():
        return s.solve(method=args.solver, rtol=args.rtol, maxit=args.maxit,
                       restart=args.restart if args.solver == "gmres" else 2, callback=progress)

    for i in range(args.warmup):
        log(f"warmup solve {i + 1}/{args.warmup}")
        one_solve()
    torch.cuda.synchronize()
    s.profile_enable(True)
    infos = []
    log(f"timing {args.steps} solve(s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x, info = one_solve()
        infos.append(info)
        log(f"solve {i + 1}: {info['iters']} iterations, {info['applies']} applies, "
            f"rel_res {info['rel_res']:.3e}, {info['seconds']:.2f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile_enable(False)
    helm = s.helmholtz_residual(x)

    applies = sum(i["applies"] for i in infos)
    pts = applies * pts_per_apply
    value = pts / elapsed / 1e9
    launch_us = prof["ms"] / prof["launches"] * 1e3
    bytes_per_launch = prof["bytes"] / prof["launches"]
    achieved = bytes_per_launch / (launch_us * 1e-6) / 1e9
    kname = {"blocked_2d": "block_steps_kernel", "blocked_3d": "block3d_steps_kernel",
             "node": "step_kernel"}.get(tun["kernel"], tun["kernel"])

    result = {
        "metric": "grid-pt updates/s (GPts/s, % HBM roofline) + time to Helmholtz residual 1e-8",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-state/f64-acc",
        "data": "synthetic (seeded random c^2 and Gaussian sources)",
        "config": {
            "workload": f"square {args.n}^2, order {order}, random c^2 in [0.5,2], omega=200, 4 Gaussian sources, "
                        + (f"GMRES({args.restart})" if args.solver == "gmres" else "CG (1/c^2 inner product)")
                        + f" to {args.rtol:g}",
            "n": args.n, "order": order, "omega": w["omega"], "nt": tp["nt"], "solver": args.solver,
            "restart": args.restart if args.solver == "gmres" else None,
            "rtol": args.rtol, "precision": args.precision, "kernel": tun["kernel"], "steps_per_launch": kblock,
            "tile_rows": tun["tile"], "owned_tile": [tile_x, tile_y],
        },
        "time_to_residual_s": round(elapsed / args.steps, 4),
        "converged": all(i["converged"] for i in infos),
        "rel_res": infos[-1]["rel_res"],
        "helmholtz_rel_res": helm,
        "solver_iters": infos[-1]["iters"],
        "applies_per_solve": infos[-1]["applies"],
        "stepping_share": round(prof["ms"] * 1e-3 / elapsed, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, {"n": args.n, "order": order, "precision": args.precision,
                                                "kblock": tun["kblock"], "tile_rows": tun["tile"]}),
            "bytes_per_launch": bytes_per_launch,
            "launch_us": round(launch_us, 3),
            "launches": prof["launches"],
            "kernel_GPts_per_s": round(prof["point_steps"] / prof["ms"] * 1e-6, 2),
            # temporal blocking: the same rate against the one-step-per-pass
            # roofline of the timed applications (A v: no forcing, variable
            # c^2: 3 state levels + c^2 + the FP64 accumulator read and
            # written = 48 B per point-step in FP64, 166.7 GPts/s at 8 TB/s)
            "unblocked_bytes_per_point_step": unblocked_bytes(args.precision, True, False),
            "kernel_GPts_vs_unblocked_roofline": round(prof["point_steps"] / prof["ms"] * 1e-6
                                                       / (HBM_PEAK_GBS / unblocked_bytes(args.precision, True,
                                                                                          False)), 3),
        },
    }
    if args.cpu_baseline:
        log("CPU oracle baseline: one W_h(v, 0) application on the host")
        rate, cores, sec, nt = cpu_baseline(dict(w, n=args.n), order, None)
        rate1, sec1, nt1 = cpu_single_thread(dict(w, n=args.n), order)
        result["cpu_baseline"] = {
            "value": round(rate, 4), "unit": "GPts/s", "cores": cores, "kind": "oracle",
            "single_thread_value": round(rate1, 4), "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "single_thread_sample": f"{nt1} leapfrog steps of the same grid on one thread, {sec1:.1f}s",
            "sample": f"one W_h(v,0) application ({nt} leapfrog steps over {unknowns} unknowns) of the same "
                      f"workload, FP64, {sec:.1f}s; CPU time to residual extrapolated as "
                      f"{applies / args.steps} applies x {sec:.1f}s = {applies / args.steps * sec:.0f}s",
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
