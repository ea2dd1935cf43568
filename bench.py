#!/usr/bin/env python3
"""Benchmark of the MI355X memory-saving UGKS step.

Workload: the 2D hypersonic cylinder -- 20,000 unstructured cells (200 x 95
O-grid, outer 5 rings cut into triangles) around a unit cylinder in a
15-radius far field, Shakhov Pr = 2/3, Ma = 5, Kn = 0.1, isothermal wall,
60 x 60 velocity grid on [-15, 15]^2: 72 million cell-velocity updates per
step.  A step is one full time step of the scheme (macro gradients,
interface equilibria, fused sweep with wall, macro update, heat flux and
both stages of the f update) on inputs resident in HBM.

Prints one JSON line: cell-velocity updates/s; the roofline of the fused
sweep kernel (live HIP-event timing of that kernel on its stream): the
kernel is bound by the vector ALUs, so `roofline` gives the method's
algorithmic FP64 flop rate against the 78.6 TFLOP/s vector peak, with its
algorithmic HBM bandwidth against 8 TB/s and the measured HBM traffic
beside it; and the FP64 CPU oracle timed on the host on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, vector FP64


def alg_flops_per_update(dim: int, nf: float) -> float:
    """FP64 flops of one cell-velocity update in the method's minimal form:
    one limited slope per (cell, velocity) (least-squares gradient: a
    difference and dim FMAs per neighbour and component; Venkatakrishnan:
    face increment, dp^2 + eps^2, numerator, denominator, cross-multiplied
    comparison per face and component; one reciprocal by two Newton steps
    and the scaling), every face flux once (nf/2 per cell: normal velocity,
    face value and u.grad per component, the tabulated Gaussian, the
    time-integrated interface value -- about 50 flops for h and b, 30 for h
    alone -- and its accumulation), then source, stage 1, moments, heat flux
    and stage 2 (75 in 2D, 50 in 3D).  An FMA counts two."""
    nc = 2 if dim == 2 else 1
    slope = nc * (nf * (1 + 2 * dim) + nf * (2 * dim + 2 + 3 + 4 + 2) + 9 + 2 * dim)
    faces = 0.5 * nf * (2 * dim + nc * 4 * dim + 2 + (50 if nc == 2 else 30) + 1 + 2 * nc)
    return slope + faces + (75 if dim == 2 else 50)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_cylinder20k_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2412_06546_amd", "csrc", "ugks_kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(fstore: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    key = f"traffic_bytes_per_launch_{fstore}"
    return float(vals[key]) if key in vals else None


def copy_calibration(nbytes: int, reps: int):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def cpu_baseline(case, target_s: float, max_steps: int):
    """The FP64 oracle as it stands, on the host cores, on the same workload;
    set-up (time step, initial state) excluded.  Timed with all cores
    (bounded by target_s), then one step on one core."""
    import oracle
    nc, nv = len(case["mesh"]["cell_volume"]), len(case["vgrid"]["w"])
    o = oracle.Oracle(case, omp_threads=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    cores = o.threads
    steps, t = 0, 0.0
    while steps < max_steps and t < target_s:
        t0 = time.perf_counter()
        o.step(1)
        t += time.perf_counter() - t0
        steps += 1
    o.set_threads(1)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    o.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": nc * nv * steps / t, "unit": "cell-velocity updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": nc * nv / t1, "host_cpu": model, "host_logical_cpus": os.cpu_count(),
            "sample": f"{steps} full steps of the same {nc}-cell x {nv}-velocity workload on {cores} threads "
                      f"({t:.1f} s, OpenMP over cells, gcc -O2), then 1 step on 1 thread ({t1:.1f} s)"}


def run_gpu(case, fstore: str, steps: int, warmup: int, mem: str = "two-buffers", chunk: int = 0):
    import torch
    from paper_2412_06546_amd import ugks
    s = ugks.Solver(case, fstore=fstore, mem=mem, chunk=chunk)
    nc, nv, ncomp = s.nc, s.nv, s.ncomp
    s.step(warmup)
    torch.cuda.synchronize()
    s.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sweep_ms, pro_ms, n = s.profile_read()
    s.profile(False)
    W, _ = s.macros()
    bytes_per_value = {"f64": 8, "f32": 4, "bf16": 2}[fstore]
    alg_bytes = nc * nv * ncomp * bytes_per_value * 2      # read f once, write f once
    sweep_avg_s = sweep_ms / n / 1e3
    out = dict(ms_per_step=ms / steps, wall_s=wall, updates_per_s=nc * nv * steps / (ms / 1e3),
               sweep_ms_avg=sweep_ms / n, prologue_ms_avg=pro_ms / n, alg_bytes=alg_bytes,
               achieved_gbs=alg_bytes / sweep_avg_s / 1e9, footprint_bytes=s.footprint_bytes,
               finite=bool((W[:, 0] > 0).all()))
    s.close()
    return out


def run_serving(args):
    """Continuous batching of a Poisson stream of independent 2D cases: all-
    triangle cylinder meshes of 2k-50k cells, 20^2-64^2 velocity grids, Ma in
    [0.5, 6], Kn in [1e-3, 1], f in FP32 with FP64 macros, each run to a
    residual of 1e-6 or the step cap."""
    from paper_2412_06546_amd import serve
    t0 = time.perf_counter()
    reqs = serve.poisson_stream(n_cases=args.serving, rate=4.0, max_steps=args.serving_steps, fstore="f32")
    print(f"# generated {len(reqs)} cases in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    backend = serve.GpuBackend(batched=args.serving_mode == "batched")
    srv = serve.Server(int(args.serving_budget_gb * 1e9), max_active=16, chunk=20, backend=backend)
    res = srv.run(reqs)
    summ = serve.Server.summary(res)
    for r in res:
        if r.error:
            print(f"# case {r.rid} ({reqs[r.rid].case['name']}): {r.error}", file=sys.stderr, flush=True)
    line = {"metric": "serving time-to-result (p50/p99) and cell-velocity updates/s", "value": summ["p50_time_to_result_s"],
            "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": f"Poisson stream (4/s) of {len(reqs)} cylinder cases, 2k-50k triangles, "
                                   f"20^2-64^2 velocities, tol 1e-6, cap {args.serving_steps} steps, f32",
                       "mode": args.serving_mode + (" (one batched launch per kernel per round)" if
                                                    args.serving_mode == "batched" else " (a stream per case)"),
                       "budget_bytes": srv.budget, "peak_bytes": srv.peak_used},
            "serving": summ}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fstore", choices=["f64", "f32", "bf16"], default="f64")
    ap.add_argument("--workload", choices=["cylinder", "sphere", "spherehex", "liftingbody"], default="cylinder",
                    help="cylinder: the 2D benchmark; sphere: the 3D sphere (50,688 tetrahedra x 24^3 velocities); "
                         "spherehex: the same shell as 50,688 hexahedra; "
                         "liftingbody: the X38-sized case (1,058,685 cells x 4,548 velocities, no CPU baseline)")
    ap.add_argument("--mem", choices=["two-buffers", "in-place"], default="two-buffers",
                    help="f in two buffers (f^n, f^{n+1}) or one buffer updated in place by velocity chunks")
    ap.add_argument("--chunk", type=int, default=0, help="in-place mode: velocities per chunk (0 = the library default, 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other f storage precision")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serving", type=int, default=0, metavar="N",
                    help="instead: serve a Poisson stream (4/s) of N cylinder cases and report p50/p99")
    ap.add_argument("--serving-steps", type=int, default=400, help="step cap per served case")
    ap.add_argument("--serving-budget-gb", type=float, default=200.0)
    ap.add_argument("--serving-mode", choices=["batched", "streams"], default="batched")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(velocity-space sharding over RCCL is a design, not code). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, 5)
        return
    if args.serving:
        run_serving(args)
        return

    from paper_2412_06546_amd import cases
    case = {"cylinder": cases.case_cylinder, "sphere": cases.case_sphere,
            "spherehex": lambda: cases.case_sphere(n=16, n_r=33, kind="hex"),
            "liftingbody": cases.case_lifting_body}[args.workload]()
    nc, nv = len(case["mesh"]["cell_volume"]), len(case["vgrid"]["w"])
    print(f"# workload {case['name']}: {nc} cells x {nv} velocities, f {args.fstore}", file=sys.stderr, flush=True)
    main_run = run_gpu(case, args.fstore, args.steps, args.warmup, args.mem, args.chunk)
    print(f"# gpu {args.fstore}: {main_run['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    other = []
    if not args.no_secondary:
        for fs2 in [x for x in ("f64", "f32", "bf16") if x != args.fstore]:
            r2 = run_gpu(case, fs2, max(5, args.steps // 2), args.warmup, args.mem, args.chunk)
            other.append({"f_storage": fs2, "value": r2["updates_per_s"], "ms_per_step": r2["ms_per_step"],
                          "sweep_ms": r2["sweep_ms_avg"], "achieved_gbs": r2["achieved_gbs"]})
            print(f"# gpu {fs2}: {r2['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    traffic = measured_traffic(args.fstore) if args.workload == "cylinder" and args.mem == "two-buffers" else None
    # the sweep is bound by the vector ALUs (about 73 % busy, profiles/k_sweep_cylinder20k_valu.txt), not by HBM
    dim = int(case["mesh"]["dim"])
    nf_avg = float(np.bincount(np.concatenate([case["mesh"]["face_cells"][:, 0],
                                               case["mesh"]["face_cells"][:, 1][case["mesh"]["face_cells"][:, 1] >= 0]]),
                               minlength=nc).mean())
    fpu = alg_flops_per_update(dim, nf_avg)
    alg_flops = fpu * nc * nv
    tflops = alg_flops / (main_run["sweep_ms_avg"] / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "k_sweep" if args.mem == "two-buffers" else "k_sweep_chunk (every chunk) + k_sweep_finish",
                "kernel_ms": round(main_run["sweep_ms_avg"], 4),
                "alg_flops_per_update": round(fpu, 1), "alg_flops_per_launch": alg_flops,
                "hbm": {"achieved": round(main_run["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(main_run["achieved_gbs"] / HBM_PEAK_GBS, 4),
                        "alg_bytes_per_launch": main_run["alg_bytes"],
                        "traffic_gbs": round(traffic / (main_run["sweep_ms_avg"] / 1e3) / 1e9, 1) if traffic else None}}
    line = {
        "metric": "cell-velocity updates/s",
        "value": main_run["updates_per_s"],
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.fstore,
        "data": "synthetic",
        "config": {"workload": f"{case['name']}: " + {
                       "cylinder": "2D hypersonic cylinder Ma 5 Kn 0.1 Shakhov, isothermal wall",
                       "sphere": "3D sphere Ma 4 Kn 0.05 Shakhov, isothermal wall",
                       "spherehex": "3D sphere (hexahedra) Ma 4 Kn 0.05 Shakhov, isothermal wall",
                       "liftingbody": "3D X38-sized lifting body Ma 8 AoA 20 Kn 0.01 Shakhov, wall 5.39 T_inf, "
                                      "unstructured velocity set"}[args.workload],
                   "n_cells": nc, "n_vel": nv, "f_storage": args.fstore, "macros": "f64", "mem": args.mem,
                   "prologue_ms": round(main_run["prologue_ms_avg"], 4),
                   "footprint_bytes": main_run["footprint_bytes"]},
        "roofline": roofline,
    }
    if args.mem == "in-place":
        from paper_2412_06546_amd.ugks import UGKS_DEFAULT_CHUNK
        line["config"]["chunk"] = min(args.chunk if args.chunk > 0 else UGKS_DEFAULT_CHUNK, nv)
    if other:
        line["other_precision"] = other
    if not args.no_cpu_baseline and args.workload != "liftingbody":
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds, 5)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
