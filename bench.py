#!/usr/bin/env python3
"""Benchmark of the MI355X memory-saving UGKS step.

Headline workload: the X38-sized synthetic lifting body -- 1,058,685
hexahedra and prisms around a blunt lifting body, Ma 8 at 20 degrees angle
of attack, Kn 0.01, Shakhov Pr 0.72, isothermal wall at 5.39 T_inf,
unstructured (octree) velocity mesh of 4,548 points, f in FP64: 4.81e9
cell-velocity updates per step, the size of the paper's only timed workload
(Section 4.3, Table UGKSeff) and the largest single-GPU configuration.  A
step is one full time step of the scheme (macro gradients, interface
equilibria, fused sweep with wall, macro update, heat flux and both stages
of the f update) on inputs resident in HBM.  The sweep is the unordered push
(--sweep push_unordered: every face flux once, by its upwind cell, all cells
in one launch in stored order; sums rounded in no fixed order); the
deterministic coloured push is timed beside it.

Prints one JSON line:
  value      cell-velocity updates/s of the headline (HIP events on the
             library's stream around the timed steps);
  roofline   the sweep against the roof that binds it: the algorithmic
             bytes (f read once and written once per update: 2 n_comp s
             bytes) at 8 TB/s and the method's algorithmic FP64 flops at
             78.6 TFLOP/s give two least times, the longer one is the bound
             (the vector ALUs for the lifting body: 22.7 flops per byte,
             past the ridge of 9.8); achieved = algorithmic flops (or bytes)
             over the sweep's average duration (HIP events recorded by the
             library around every sweep launch); both figures beside; the
             measured HBM traffic from the committed counter profile (when
             the kernel source and sweep are the ones profiled);
  coloured_push   the headline step with the coloured (bitwise
             reproducible) push sweep;
  other_precision   the same workload with f in FP32 and BF16;
  secondary_workloads   the 2D cylinder (20,000 cells x 3,600 velocities);
  serving    a bounded serving leg: a Poisson stream of 16 small 2D cases
             (supersonic cylinders, FP64 f) each run to a relative residual
             of 1e-6 (cap 60,000 steps): converged and capped counts, p50/p99
             time-to-converged, updates/s;
  cpu_baseline   the FP64 CPU oracle on the host cores on a bounded sample of
             the lifting body (same velocity set and cell types, fewer cells).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, vector FP64
KERNEL_SRC = os.path.join(ROOT, "paper_2412_06546_amd", "csrc", "ugks_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
DEFAULT_SWEEP = "push_unordered"
TRAFFIC_FILES = {"liftingbody": os.path.join(PROFILES, "k_push_sweep_liftingbody1m_traffic.txt"),
                 "cylinder": os.path.join(PROFILES, "k_push_sweep_cylinder20k_traffic.txt")}

WORKLOADS = {
    "liftingbody": "3D X38-sized lifting body Ma 8 AoA 20 Kn 0.01 Shakhov Pr 0.72, wall 5.39 T_inf, "
                   "unstructured (octree) velocity set",
    "cylinder": "2D hypersonic cylinder Ma 5 Kn 0.1 Shakhov Pr 2/3, isothermal wall",
    "sphere": "3D sphere (tetrahedra) Ma 4 Kn 0.05 Shakhov Pr 0.72, isothermal wall",
    "spherehex": "3D sphere (hexahedra) Ma 4 Kn 0.05 Shakhov Pr 0.72, isothermal wall",
}


def make_case(workload: str):
    from paper_2412_06546_amd import cases
    return {"cylinder": cases.case_cylinder, "sphere": cases.case_sphere,
            "spherehex": lambda: cases.case_sphere(n=16, n_r=33, kind="hex"),
            "liftingbody": cases.case_lifting_body}[workload]()


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


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload: str, fstore: str, path: str | None = None, sweep: str | None = None):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary of this workload, or None when there is none, the kernel
    source changed since it was taken or it was taken with another sweep."""
    path = path or TRAFFIC_FILES.get(workload)
    if not path or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if sweep is not None and vals.get("sweep") != sweep:
        return None
    key = f"traffic_bytes_per_launch_{fstore}"
    return float(vals[key]) if key in vals else None


def mean_faces_per_cell(case) -> float:
    fc = np.asarray(case["mesh"]["face_cells"])
    nc = len(case["mesh"]["cell_volume"])
    return float(np.bincount(np.concatenate([fc[:, 0], fc[:, 1][fc[:, 1] >= 0]]), minlength=nc).mean())


def copy_calibration(nbytes: int, reps: int):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(target_s: float):
    """The FP64 oracle as it stands, on the host cores.  The full lifting
    body (38.5 GB of f, about a minute per step on 16 cores) is beyond a
    bounded run, so the sample is a cut-down of the same workload: the same
    4,548-point velocity set, hexahedra and prisms, wall and far field,
    64,920 cells (16 x 16 points per cube face, 40 layers), timed over whole
    steps on all cores up to target_s; then a smaller cut-down (8 x 8 points,
    20 layers: 7,830 cells) for one step on one core.  Set-up (time step,
    initial state) excluded."""
    import oracle
    from paper_2412_06546_amd import cases
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    case = cases.case_lifting_body(n=16, n_r=40, n_prism_columns=87)
    nc, nv = len(case["mesh"]["cell_volume"]), len(case["vgrid"]["w"])
    o = oracle.Oracle(case, omp_threads=threads)
    cores = o.threads
    steps, t = 0, 0.0
    while steps < 8 and t < target_s:
        t0 = time.perf_counter()
        o.step(1)
        t += time.perf_counter() - t0
        steps += 1
    del o
    small = cases.case_lifting_body(n=8, n_r=20, n_prism_columns=21)
    nc1 = len(small["mesh"]["cell_volume"])
    o1 = oracle.Oracle(small, omp_threads=1)
    t0 = time.perf_counter()
    o1.step(1)
    t1 = time.perf_counter() - t0
    del o1
    oracle.lib().orc_set_threads(cores)
    return {"value": nc * nv * steps / t, "unit": "cell-velocity updates/s", "cores": cores, "kind": "oracle",
            "single_core_value": nc1 * nv / t1, "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": f"{steps} full steps of a {nc}-cell cut-down of the lifting body (same 4,548-velocity set, "
                      f"hexahedra and prisms, wall and far field) on {cores} threads ({t:.1f} s, OpenMP over "
                      f"cells, gcc -O2); then 1 step of a {nc1}-cell cut-down on 1 thread ({t1:.1f} s)"}


def run_gpu(case, fstore: str, steps: int, warmup: int, mem: str = "two-buffers", chunk: int = 0,
            sweep: str = "auto"):
    """Warm-up steps, then exactly `steps` timed steps between device
    synchronisations; HIP events on torch's current stream (the stream the
    library launches on) around the timed steps, and the library's own
    events around every sweep launch."""
    import torch
    from paper_2412_06546_amd import ugks
    s = ugks.Solver(case, fstore=fstore, mem=mem, chunk=chunk, sweep=sweep)
    nc, nv, ncomp = s.nc, s.nv, s.ncomp
    if warmup:
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
               bytes_per_update=ncomp * bytes_per_value * 2,
               achieved_gbs=alg_bytes / sweep_avg_s / 1e9, footprint_bytes=s.footprint_bytes,
               finite=bool(np.isfinite(W).all() and (W[:, 0] > 0).all()), nc=nc, nv=nv, sweep=s.sweep,
               n_colours=s.n_colours)
    s.close()
    return out


def json_safe(x):
    """NaN (a percentile of no cases) as null: JSON has no NaN."""
    if isinstance(x, float) and x != x:
        return None
    if isinstance(x, dict):
        return {k: json_safe(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [json_safe(v) for v in x]
    return x


def sweep_kernels(run, mem):
    """The kernels one timed sweep launch consists of."""
    if run.get("sweep") == "push_unordered":
        launches = "one launch of k_push_pf (k_push) over all cells in stored order"
    else:
        launches = f"{run.get('n_colours')} colour launches of k_push_pf (k_push)"
    if mem == "in-place" and run.get("sweep", "").startswith("push"):
        return (f"push sweep in place: k_push_wall, then per velocity chunk k_push_chunk_turn and {launches}, "
                f"a last k_push_chunk_turn, k_push_final_inplace, timed together")
    if mem == "in-place":
        return "k_sweep_chunk (every chunk) + k_sweep_finish"
    if run.get("sweep", "").startswith("push"):
        return f"push sweep: k_push_wall, {launches}, k_push_final_r (k_push_final), timed together"
    return "k_sweep_pf (k_sweep)"


def roofline_of(case, run, workload, fstore, mem):
    """The sweep against the roof that binds it.  The algorithmic bytes at
    the HBM peak and the algorithmic FP64 flops at the vector peak give two
    least times for one sweep; the longer one is the bound ("alu" where the
    method's flops per byte exceed the ridge of 9.8, "hbm" below it), its
    figures at the top level, both in full beside."""
    dim = int(case["mesh"]["dim"])
    fpu = alg_flops_per_update(dim, mean_faces_per_cell(case))
    alg_flops = fpu * run["nc"] * run["nv"]
    sweep_s = run["sweep_ms_avg"] / 1e3
    tflops = alg_flops / sweep_s / 1e12
    traffic = measured_traffic(workload, fstore, sweep=run.get("sweep")) if mem == "two-buffers" else None
    hbm = {"achieved": round(run["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(run["achieved_gbs"] / HBM_PEAK_GBS, 4), "alg_bytes_per_update": run["bytes_per_update"],
           "alg_bytes_per_launch": run["alg_bytes"]}
    alu = {"achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "alg_flops_per_update": round(fpu, 1),
           "alg_flops_per_launch": alg_flops}
    t_hbm = run["alg_bytes"] / (HBM_PEAK_GBS * 1e9)
    t_alu = alg_flops / (FP64_PEAK_TFLOPS * 1e12)
    bound = "alu" if t_alu > t_hbm else "hbm"
    top = alu if bound == "alu" else hbm
    return {"bound": bound, "achieved": top["achieved"], "peak": top["peak"], "unit": top["unit"],
            "frac": top["frac"], "traffic": traffic,
            "kernel": sweep_kernels(run, mem),
            "kernel_ms": round(run["sweep_ms_avg"], 4),
            "least_ms": {"hbm": round(t_hbm * 1e3, 4), "alu": round(t_alu * 1e3, 4)},
            "traffic_over_algorithmic": round(traffic / run["alg_bytes"], 3) if traffic else None,
            "hbm": hbm, "alu": alu}


def run_serving_leg(n_cases: int, max_steps: int, mode: str):
    """The bounded serving leg: a Poisson stream of small 2D cases (2k-5k
    triangles and quadrilaterals, 20^2-32^2 velocities, Ma 1.5-3, Kn
    0.05-1, FP64 f), each run to a residual of 1e-6 of its first step's or
    the step cap, continuous batching under an HBM budget."""
    from paper_2412_06546_amd import serve
    reqs = serve.converging_stream(n_cases=n_cases, max_steps=max_steps)
    backend = serve.GpuBackend(batched=mode == "batched")
    srv = serve.Server(int(40e9), max_active=16, chunk=50, backend=backend)
    res = srv.run(reqs)
    summ = serve.Server.summary(res)
    summ["workload"] = (f"Poisson stream (8/s) of {len(reqs)} cylinder cases, 2k-5k cells, 20^2-32^2 velocities, "
                        f"Ma 1.5-3, Kn 0.05-1, tol 1e-6, cap {max_steps} steps, f64")
    summ["mode"] = mode
    summ["peak_bytes"] = srv.peak_used
    for r in res:
        if r.error:
            print(f"# serving case {r.rid}: {r.error}", file=sys.stderr, flush=True)
    return summ


def run_serving_stream(args):
    """--serving N: the full serving configuration (a Poisson stream of N
    2D cylinder cases, 2k-50k triangles, 20^2-64^2 velocities)."""
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
    line = {"metric": "serving time-to-converged (p50/p99) and cell-velocity updates/s",
            "value": summ["p50_time_to_converged_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
            "data": "synthetic",
            "config": {"workload": f"Poisson stream (4/s) of {len(reqs)} cylinder cases, 2k-50k triangles, "
                                   f"20^2-64^2 velocities, tol 1e-6, cap {args.serving_steps} steps, f32",
                       "mode": args.serving_mode, "budget_bytes": srv.budget, "peak_bytes": srv.peak_used},
            "serving": summ}
    print(json.dumps(json_safe(line)), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fstore", choices=["f64", "f32", "bf16"], default="f64")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="liftingbody")
    ap.add_argument("--mem", choices=["two-buffers", "in-place"], default="two-buffers",
                    help="f in two buffers (f^n, f^{n+1}) or one buffer updated in place by velocity chunks")
    ap.add_argument("--chunk", type=int, default=0, help="in-place mode: velocities per chunk (0 = the library default)")
    ap.add_argument("--sweep", choices=["auto", "gather", "push", "push_unordered"], default=DEFAULT_SWEEP,
                    help="how the sweep evaluates the face fluxes (UGKS_SWEEP_*)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the coloured push, the other precisions and workloads")
    ap.add_argument("--no-serving", action="store_true", help="skip the bounded serving leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serving-leg-cases", type=int, default=16)
    ap.add_argument("--serving-leg-steps", type=int, default=60000)
    ap.add_argument("--serving-leg-mode", choices=["batched", "streams"], default="streams",
                    help="serving leg: batched steps on one stream, or a stream per case (measured the faster)")
    ap.add_argument("--serving", type=int, default=0, metavar="N",
                    help="instead: serve a Poisson stream (4/s) of N cylinder cases (2k-50k cells) and report p50/p99")
    ap.add_argument("--serving-steps", type=int, default=400, help="step cap per served case (--serving)")
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
        run_serving_stream(args)
        return

    case = make_case(args.workload)
    nc, nv = len(case["mesh"]["cell_volume"]), len(case["vgrid"]["w"])
    print(f"# workload {case['name']}: {nc} cells x {nv} velocities, f {args.fstore}", file=sys.stderr, flush=True)
    main_run = run_gpu(case, args.fstore, args.steps, args.warmup, args.mem, args.chunk, args.sweep)
    print(f"# gpu {args.fstore}: {main_run['ms_per_step']:.3f} ms/step, sweep {main_run['sweep_ms_avg']:.3f} ms",
          file=sys.stderr, flush=True)
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
        "config": {"workload": f"{case['name']}: {WORKLOADS[args.workload]}",
                   "n_cells": nc, "n_vel": nv, "f_storage": args.fstore, "macros": "f64", "mem": args.mem,
                   "prologue_ms": round(main_run["prologue_ms_avg"], 4),
                   "footprint_bytes": main_run["footprint_bytes"], "all_cells_physical": main_run["finite"],
                   "sweep": main_run["sweep"], "sweep_launches": main_run["n_colours"]},
        "roofline": roofline_of(case, main_run, args.workload, args.fstore, args.mem),
    }
    # the targets this build measures against, stated beside the figures
    line["targets"] = {
        "hbm_fraction": {"target": 0.60, "measured": line["roofline"]["hbm"]["frac"],
                         "met": line["roofline"]["hbm"]["frac"] >= 0.60},
    }
    if main_run["sweep"] == "push_unordered" and not args.no_secondary:
        # the same step with the deterministic (coloured) push sweep, beside it
        r2 = run_gpu(case, args.fstore, max(4, args.steps // 2), min(args.warmup, 2), args.mem, args.chunk, "push")
        line["coloured_push"] = {"sweep": r2["sweep"], "colour_launches": r2["n_colours"],
                                 "value": r2["updates_per_s"], "ms_per_step": r2["ms_per_step"],
                                 "sweep_ms": round(r2["sweep_ms_avg"], 4),
                                 "unordered_speedup": round(r2["ms_per_step"] / main_run["ms_per_step"], 3)}
        print(f"# gpu {args.fstore} coloured push: {r2['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if args.mem == "in-place":
        from paper_2412_06546_amd.ugks import UGKS_DEFAULT_CHUNK
        line["config"]["chunk"] = min(args.chunk if args.chunk > 0 else UGKS_DEFAULT_CHUNK, nv)
    if not args.no_secondary:
        other = []
        for fs2 in [x for x in ("f64", "f32", "bf16") if x != args.fstore]:
            r2 = run_gpu(case, fs2, max(4, args.steps // 2), min(args.warmup, 2), args.mem, args.chunk, args.sweep)
            other.append({"f_storage": fs2, "sweep": r2["sweep"], "value": r2["updates_per_s"], "ms_per_step": r2["ms_per_step"],
                          "sweep_ms": round(r2["sweep_ms_avg"], 4), "alg_gbs": round(r2["achieved_gbs"], 1),
                          "speedup_over_headline": round(main_run["ms_per_step"] / r2["ms_per_step"], 3)})
            print(f"# gpu {fs2}: {r2['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        line["other_precision"] = other
        if args.fstore == "f64":
            sp = next(o["speedup_over_headline"] for o in other if o["f_storage"] == "f32")
            line["targets"]["fp32_speedup_over_fp64"] = {"target": 1.7, "measured": sp, "met": sp >= 1.7}
        sec = []
        for wl in [w for w in ("liftingbody", "cylinder") if w != args.workload]:
            c2 = make_case(wl)
            entry = {"workload": f"{c2['name']}: {WORKLOADS[wl]}"}
            for fs2 in ("f64", "f32"):
                r2 = run_gpu(c2, fs2, max(20, args.steps), 3, sweep=args.sweep)
                rl = roofline_of(c2, r2, wl, fs2, "two-buffers")
                entry[fs2] = {"value": r2["updates_per_s"], "sweep": r2["sweep"], "ms_per_step": round(r2["ms_per_step"], 4),
                              "sweep_ms": rl["kernel_ms"], "bound": rl["bound"], "hbm_frac": rl["hbm"]["frac"],
                              "alu_frac": rl["alu"]["frac"],
                              "traffic": rl["traffic"]}
                print(f"# gpu {wl} {fs2}: {r2['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
            entry["f32_speedup_over_f64"] = round(entry["f64"]["ms_per_step"] / entry["f32"]["ms_per_step"], 3)
            sec.append(entry)
            del c2
        line["secondary_workloads"] = sec
    if not args.no_serving:
        print("# serving leg ...", file=sys.stderr, flush=True)
        line["serving"] = run_serving_leg(args.serving_leg_cases, args.serving_leg_steps, args.serving_leg_mode)
    if not args.no_cpu_baseline and args.workload == "liftingbody":
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(json_safe(line)), flush=True)


if __name__ == "__main__":
    main()
