#!/usr/bin/env python3
"""Throughput of the direct Poisson solver on one MI355X.

A step is one whole solve of L_h p = f (eq. (poi), Section 2) on the
1024 x 512 x 384 channel slab (periodic x and y, Neumann walls in z on a
tanh-stretched grid, rhs = divergence of a seeded random staggered
velocity): FP32 transforms, FP64 z elimination and FP64 iterative refinement
to a relative residual of 1e-10, including the final residual check.  The
plain FP64 solve of the same rhs is timed beside it.  Inputs sit in HBM
before the timed region.

Printed: one JSON line with grid points per second, the roofline position of
the dominant kernel (algorithmic bytes / its HIP-event-timed duration), and
the CPU oracle's rate on a bounded sample of the same grid.

    python bench.py [--steps K] [--warmup W] [--config c3] [--gpus 1]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Poisson grid pts/s, FP64 vs FP32+refine at 1e-10 residual; achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0

# kernels of one refinement-mode solve: debug stage, name, algorithmic bytes
# per grid point (each reads and writes the field once in its precision)
KERNELS32 = [
    (1, "x_fwd (f64 in, f32 out)", 12),
    (2, "y_fwd f32", 8),
    (3, "z_solve (f64 arithmetic, f32 io)", 8),
    (4, "y_inv f32", 8),
    (5, "x_inv (f32 in, f64 out)", 12),
    (6, "residual+x_fwd (p, f f64 in; f32 out)", 20),
    (7, "x_inv+update (f32 + p in, p out)", 20),
    (8, "residual norm (p, f f64 in)", 16),
]
KERNELS64 = [
    (1, "x_fwd f64", 16),
    (2, "y_fwd f64", 16),
    (3, "z_solve f64", 16),
    (4, "y_inv f64", 16),
    (5, "x_inv f64", 16),
]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def time_solves(plan, fd, pd, steps, warmup, torch):
    for _ in range(warmup):
        plan.solve(fd, pd)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    s.record()
    for _ in range(steps):
        plan.solve(fd, pd)
    e.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return s.elapsed_time(e) / steps, wall


def time_stage(plan, stage, a, b, reps, torch):
    """Average duration of one kernel launch, HIP events on the launch stream."""
    plan.debug_stage(stage, a, b)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        plan.debug_stage(stage, a, b)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c3.txt")


def source_digest() -> str:
    """Hash of the kernel sources (paper_2001_05234_amd/csrc), so counter
    readings taken with other kernels are not reported as current."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2001_05234_amd", "csrc")
    for n in sorted(os.listdir(d)):
        if n.endswith((".h", ".hip")):
            h.update(n.encode())
            with open(os.path.join(d, n), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    by a device copy) from the committed counter summary, or None when there is
    none or it was taken with other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [l.rstrip("\n") for l in fh if l.strip() and not l.startswith("#")]
    except OSError:
        return None
    if not lines or lines[0] != "source-digest: " + source_digest():
        return None
    for l in lines[1:]:
        name, fetch, write = l.split("\t")
        if name == kernel:
            return float(fetch) + float(write)
    return None


def workload_text(name, pr, xform_x):
    """What is solved: sizes, boundary pairs, grid and rhs of the problem."""
    import numpy as np

    code = ["P", "N", "D", "Fd", "Fn"]  # Fd / Fn: Dirichlet / Neumann face of a face-located field
    bc = "/".join(code[pr.bc[2 * a]] + code[pr.bc[2 * a + 1]] for a in range(3))
    grid = "uniform z" if np.allclose(pr.dzf, pr.dzf[0]) else "tanh-stretched z (a=1.5)"
    rhs = ("divergence of a seeded N(0,1) staggered velocity" if pr.rhs_kind == "divergence"
           else "seeded U[-1,1]" + (", projected" if all(b in (0, 1) for b in pr.bc) else ""))
    xf = {"auto": "FFT", "fft": "FFT", "dense": "dense split-bf16 matrix-core"}[xform_x]
    return (f"{name}: {pr.nx}x{pr.ny}x{pr.nz}, bc {bc}, {grid}, rhs {rhs}; FP32 transforms ({xf} x), "
            f"FP64 Thomas + residual, refined to rel. residual 1e-10")


def run_stage(plan, stage, fd, pd, a32, reps, torch):
    """One kernel of the refinement plan in the order of a solve (reps = 0:
    a single untimed launch).  Stages 6 and 8 test the residual of pd, so the
    finished flag is cleared first."""
    if stage in (6, 8):
        plan.debug_stage(0, fd, pd)
    a, b = (fd, pd) if stage in (1, 6, 8) else (fd, a32)
    if reps == 0:
        plan.debug_stage(stage, a, b)
        return 0.0
    return time_stage(plan, stage, a, b, reps, torch)


def copy_gbs(torch, nbytes):
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(10):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / 10
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def bench_project(torch, capi, pr, args):
    """The projection step on the config's grid: seeded N(0,1) staggered
    velocity (zero on wall faces) and pressure drawn on the device, gdt =
    1.6e-3, FP64.  Byte model per point: divergence fused into the x
    transform 24 + 8, the y, z, y and x sweeps 4 x 16, the correction
    40 + 32: 168 B."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(pr.seed + 2000)
    fields = []
    for a in range(4):
        x = torch.randn((pr.nz, pr.ny, pr.nx), dtype=torch.float64, device="cuda", generator=gen)
        if a < 3 and pr.bc[2 * a] != 0:  # wall: the last face of a bounded axis
            idx = [slice(None)] * 3
            idx[2 - a] = -1
            x[tuple(idx)] = 0.0
        fields.append(x)
    plan = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp64",
                     autotune=not args.no_autotune)
    for _ in range(args.warmup):
        plan.project(*fields, 1.6e-3)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(args.steps):
        plan.project(*fields, 1.6e-3)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / args.steps
    # the same step with the implicit-diffusion pressure update (alpha =
    # gamma nu dt / 2, nu = 2e-4) and the time-step bound of eq. (dt) on the
    # corrected velocity (one more pass reading u, v, w: 24 B per point)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    alpha = 0.5 * 1.6e-3 * 2e-4
    for _ in range(args.warmup):
        plan.project_ex(*fields, 1.6e-3, alpha=alpha, nu=2e-4, dt_max=dt)
    torch.cuda.synchronize()
    s.record()
    for _ in range(args.steps):
        plan.project_ex(*fields, 1.6e-3, alpha=alpha, nu=2e-4, dt_max=dt)
    e.record()
    torch.cuda.synchronize()
    ms_ex = s.elapsed_time(e) / args.steps
    plan.close()
    return {"projection_ms_per_step": ms, "grid_pts_per_s": pr.npts / (ms * 1e-3),
            "algorithmic_GBps": 168 * pr.npts / (ms * 1e-3) / 1e9, "bytes_per_point": 168,
            "implicit_update_and_dt_ms_per_step": ms_ex, "dt_max": float(dt.item()),
            "grid": [pr.nx, pr.ny, pr.nz], "steps": args.steps}


def bench_batched(torch, capi, inputs, args):
    """64 uneven problems (sizes, boundary sets and stretching drawn from a
    seed) solved as one graph launch, FP32 transforms + FP64 refinement."""
    probs = inputs.batch_c5()
    fs = [torch.from_numpy(pr.rhs()).cuda() for pr in probs]
    ps = [torch.zeros_like(f) for f in fs]
    plan = capi.BatchedPlan(probs, precision="fp32_refine", tol=1e-10, max_iter=4, autotune=not args.no_autotune)
    for _ in range(3):
        plan.solve(fs, ps)
    torch.cuda.synchronize()
    # every batch timed on its own (events around each graph launch), and the
    # whole run once: mean, min and median per batch
    reps = max(20, args.steps)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for a, b in ev:
        a.record()
        plan.solve(fs, ps)
        b.record()
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    each = sorted(a.elapsed_time(b) for a, b in ev)
    ms_min, ms_med = each[0], each[len(each) // 2]
    npts = sum(pr.npts for pr in probs)
    conv = all(plan.info(i)["converged"] for i in range(len(probs)))
    worst = max(plan.info(i)["residual"] for i in range(len(probs)))
    plan.close()
    say(f"[bench] batched: {len(probs)} problems, {npts} points, {ms:.3f} ms (min {ms_min:.3f}, median "
        f"{ms_med:.3f}), converged {conv}, worst residual {worst:.2e}")
    return {"workload": "c5: 64 uneven problems, seed 5, FP32 transforms + FP64 refinement to 1e-10, one graph "
                        "launch of grouped kernels",
            "value": npts / (ms * 1e-3), "unit": "grid pts/s", "ms_per_step": ms, "ms_min": ms_min,
            "ms_median": ms_med, "reps": reps, "grid_points": npts, "converged": conv, "worst_residual": worst}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, f, nz_sample, nz_sample_1t):
    """The oracle, as it stands, on the first nz_sample z-levels of the grid
    (full x-y planes: the same per-point work, O(nx + ny) transform
    multiply-adds plus the z elimination), with all its OpenMP threads; then
    on one thread over the first nz_sample_1t levels."""
    import numpy as np

    from oracle import oracle

    def run(nzs):
        fs = np.ascontiguousarray(f[:nzs])
        dzs = np.ascontiguousarray(pr.dzf[:nzs])
        t0 = time.perf_counter()
        oracle.solve(fs, pr.bc, pr.dx, pr.dy, dzs)
        return fs.size, time.perf_counter() - t0

    threads = oracle.threads()
    pts, dt = run(nz_sample)
    oracle.set_threads(1)
    pts1, dt1 = run(nz_sample_1t)
    oracle.set_threads(threads)
    return {"value": pts / dt, "unit": "grid pts/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle solve (O(N^2) transforms + Thomas) of the first {nz_sample} of "
                      f"{pr.nz} z-levels of the {pr.nx}x{pr.ny}x{pr.nz} grid, {pts} points, {dt:.1f} s "
                      f"on {threads} OpenMP threads",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "value_1thread": pts1 / dt1,
            "sample_1thread": f"first {nz_sample_1t} z-levels, {pts1} points, {dt1:.1f} s on 1 thread"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--cpu-sample-levels", type=int, default=384)
    ap.add_argument("--cpu-sample-levels-1t", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="built-in tile choice instead of plan-time tuning")
    ap.add_argument("--solve-only", action="store_true", help="time the refine solve only (profiling runs)")
    ap.add_argument("--fp64-only", action="store_true", help="time the FP64 solve only (profiling runs)")
    ap.add_argument("--copy-only", action="store_true",
                    help="1 GiB device-to-device copies only (calibrates the HBM byte counters)")
    ap.add_argument("--kernel-only", type=int, default=0, metavar="STAGE",
                    help="time one kernel (debug stage of the refinement plan, or of the FP64 plan with "
                         "--fp64-only) exactly as the full run times it, nothing else (profiling runs)")
    ap.add_argument("--batched-only", action="store_true", help="time the 64-problem batch only (profiling runs)")
    ap.add_argument("--graph", action="store_true",
                    help="plans replay each solve as one recorded HIP graph (cans_opts.graph)")
    ap.add_argument("--xform-x", default="auto", choices=["auto", "fft", "dense"],
                    help="x transform form of the refinement plan (dense: split-bf16 matrix-core products)")
    ap.add_argument("--shift", type=float, default=0.0,
                    help="Helmholtz shift s <= 0 of (L_h + s) p = f (a side workload: with --solve-only "
                         "or --fp64-only)")
    ap.add_argument("--project", action="store_true",
                    help="time the projection step (cans_poisson_project, FP64) on the config's grid instead")
    ap.add_argument("--face-z", action="store_true",
                    help="the field on the nz-1 interior z faces of the config's grid, zero on the walls, "
                         "uniform random rhs (a side workload: with --solve-only or --fp64-only)")
    ap.add_argument("--max-iter", type=int, default=4,
                    help="most corrections the refinement plan enqueues per solve (cans_opts.max_iter); those "
                         "after convergence are launched and return at once")
    ap.add_argument("--face-x", action="store_true",
                    help="the field on the nx-1 interior x faces of the config's grid with walls in x (DST-I "
                         "along x), uniform random rhs (a side workload: with --solve-only or --fp64-only)")
    args = ap.parse_args()
    if (args.shift != 0.0 or args.face_z or args.face_x) and not (args.solve_only or args.fp64_only):
        ap.error("--shift, --face-z and --face-x time side workloads: add --solve-only or --fp64-only")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2001_05234_amd import capi, inputs

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.copy_only:
        print(json.dumps({"copy_GBps": copy_gbs(torch, 1 << 30), "bytes_per_copy": 2 * (1 << 30)}), flush=True)
        return
    capi.load()
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(torch, capi, inputs, args)}), flush=True)
        return
    # the batch first: after the large solves below have run in the process,
    # the same batch was measured 30-40 % slower (it persists after their
    # memory is freed), so each figure is taken in a fresh state
    batched = None
    if not (args.no_batched or args.solve_only or args.fp64_only or args.kernel_only or args.project):
        batched = bench_batched(torch, capi, inputs, args)
    pr = inputs.config(args.config)
    if args.project:
        print(json.dumps(bench_project(torch, capi, pr, args)), flush=True)
        return
    if args.face_z:
        # the wall-normal velocity's grid: the interior faces of the config's
        # cells (the nz cell widths stay the plan's dz)
        pr = dataclasses.replace(pr, nz=pr.nz - 1, bc=tuple(pr.bc[:4]) + (3, 3), rhs_kind="uniform",
                                 seed=pr.seed + 1000)
    if args.face_x:
        # a velocity component on the x faces of the config's cells, between
        # walls in x (zero on them): nx-1 unknowns, a DST-I of 2nx-real lines
        pr = dataclasses.replace(pr, nx=pr.nx - 1, bc=(3, 3) + tuple(pr.bc[2:]), rhs_kind="uniform",
                                 seed=pr.seed + 2000)
    say(f"[bench] generating {args.config} rhs {pr.nx}x{pr.ny}x{pr.nz}")
    f = pr.rhs()
    fd = torch.from_numpy(f).cuda()
    pd = torch.zeros_like(fd)
    npts = pr.npts

    if args.fp64_only:
        plan64 = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp64",
                           autotune=not args.no_autotune, graph=args.graph, shift=args.shift)
        if args.kernel_only:
            name = [n for s, n, _ in KERNELS64 if s == args.kernel_only][0]
            b = torch.zeros_like(fd)
            src = b if args.kernel_only == 3 else fd
            t = time_stage(plan64, args.kernel_only, src, b, max(1, args.kernel_reps // 2), torch)
            print(json.dumps({"kernel": name, "kernel_ms": t, "plan": "fp64"}), flush=True)
            return
        ms64, _ = time_solves(plan64, fd, pd, args.steps, args.warmup, torch)
        print(json.dumps({"fp64_ms_per_step": ms64, "value": npts / (ms64 * 1e-3), "shift": args.shift,
                          "face_z": args.face_z, "face_x": args.face_x, "grid": [pr.nx, pr.ny, pr.nz]}),
              flush=True)
        return
    say("[bench] fp32+refine plan")
    plan = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine",
                     tol=1e-10, max_iter=args.max_iter, autotune=not args.no_autotune, xform_x=args.xform_x,
                     graph=args.graph,
                     shift=args.shift)
    if args.kernel_only:
        # the stages before it fill the plan's spectral field as in a solve
        a32 = torch.zeros_like(fd)
        for stage, name, _ in KERNELS32:
            if stage == args.kernel_only:
                t = run_stage(plan, stage, fd, pd, a32, args.kernel_reps, torch)
                print(json.dumps({"kernel": name, "kernel_ms": t, "plan": "fp32_refine"}), flush=True)
                return
            run_stage(plan, stage, fd, pd, a32, 0, torch)
        raise SystemExit(f"no stage {args.kernel_only}")
    ms, wall = time_solves(plan, fd, pd, args.steps, args.warmup, torch)
    info = plan.info()
    say(f"[bench] refine: {ms:.3f} ms/solve, info {info}")
    if not info["converged"]:
        raise SystemExit("refinement did not reach 1e-10")
    out = {
        "metric": METRIC, "value": npts / (ms * 1e-3), "unit": "grid pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": workload_text(args.config, pr, plan.xform_mode(0)),
                   "grid_points": npts, "corrections": info["iterations"], "graph": args.graph,
                   "residual": info["residual"], "residual_inf": info["residual_inf"], "wall_s": wall},
    }
    if args.shift != 0.0 or args.face_z or args.face_x:
        out["config"].update({"shift": args.shift, "face_z": args.face_z, "face_x": args.face_x,
                              "grid": [pr.nx, pr.ny, pr.nz]})
    if args.solve_only:
        print(json.dumps(out), flush=True)
        return

    # per-kernel durations of the refinement path (HIP events on the stream)
    a32 = torch.zeros_like(fd)
    times = {}
    for stage, name, bpp in KERNELS32:
        t = run_stage(plan, stage, fd, pd, a32, args.kernel_reps, torch)
        times[stage] = t
        say(f"[bench]   {name:42s} {t:8.3f} ms  {bpp * npts / (t * 1e-3) / 1e9:8.1f} GB/s")
    nr = info["iterations"]
    # one solve converged after nr corrections: the initial solve, check 0
    # fused with the first forward x transform, then per correction y, z, y,
    # x+update and a norm-only check (plus a fused residual when not final)
    counts = {1: 1, 2: 1 + nr, 3: 1 + nr, 4: 1 + nr, 5: 1, 6: max(1, nr), 7: nr, 8: nr}
    dom = max(times, key=lambda s: counts[s] * times[s])
    dname, dbpp = [(n, b) for s, n, b in KERNELS32 if s == dom][0]
    achieved = dbpp * npts / (times[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dname) if args.config == "c3" and args.xform_x == "auto" else None
    out["roofline"] = {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                       "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                       "algorithmic_bytes_per_launch": dbpp * npts,
                       "algorithmic_bytes_per_point": dbpp, "kernel_ms": times[dom]}
    out["kernels_ms"] = {n: round(times[s], 4) for s, n, _ in KERNELS32}
    plan.close()
    del a32

    # plain FP64 solve of the same rhs
    say("[bench] fp64 plan")
    plan64 = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp64",
                       autotune=not args.no_autotune, graph=args.graph)
    ms64, _ = time_solves(plan64, fd, pd, max(1, args.steps // 2), 2, torch)
    k64 = {}
    b = torch.zeros_like(fd)
    for stage, name, bpp in KERNELS64:
        # the z stage runs in place, as in a solve (in != out would add a copy)
        src = b if stage == 3 else fd
        k64[name] = round(time_stage(plan64, stage, src, b, max(1, args.kernel_reps // 2), torch), 4)
    out["fp64"] = {"value": npts / (ms64 * 1e-3), "unit": "grid pts/s", "ms_per_step": ms64, "kernels_ms": k64}
    say(f"[bench] fp64: {ms64:.3f} ms/solve {k64}")
    plan64.close()
    del b
    del fd, pd
    # the projection step around the solve on the same grid (FP64)
    if all(pr.bc[2 * a] == pr.bc[2 * a + 1] and pr.bc[2 * a] in (0, 1) for a in range(3)):
        say("[bench] projection step")
        out["projection"] = bench_project(torch, capi, pr, argparse.Namespace(
            steps=max(5, args.steps // 2), warmup=2, no_autotune=args.no_autotune))
    out["copy_GBps"] = copy_gbs(torch, 1 << 30)
    if batched is not None:
        out["batched"] = batched

    if not args.no_cpu_baseline:
        say("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pr, f, min(args.cpu_sample_levels, pr.nz),
                                           min(args.cpu_sample_levels_1t, pr.nz))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
