"""Continuous batching of independent flow cases on one GPU.

Requests (a case, an arrival time, a residual tolerance and a step cap)
arrive over time.  A request is admitted, in arrival order, as soon as a slot
is free and its device footprint (ugks_footprint_estimate, the bytes
ugks_create will allocate) fits in what is left of the HBM budget.  The
server then advances the admitted cases in rounds: every case that is not
running gets its next chunk of steps, and all of them are enqueued together
as one batched step (ugks_batch_step: each kernel is launched once for all
these cases, its grid holding their cells end to end), so small cases fill
the GPU together and a request that arrives while others run joins the next
round.  Cases are polled without blocking (ugks_poll); a case retires when
its residual -- the L2 change of W over one step, relative to that of its
first step -- falls below the tolerance, when it reaches its step cap or
when it turns non-physical; its memory is freed and the next request
admitted.  Each case keeps its own buffers and the kernels are
deterministic, so its result in the mix equals its result alone.

A backend without step_batch gets per-case asynchronous steps instead (each
case on its own stream).  The backend is pluggable so that the scheduling
logic can be exercised without a GPU (tests use fake backends); GpuBackend
is the product path.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    case: dict
    arrival: float = 0.0       # seconds after the server starts
    tol: float = 1e-6          # stop when max_m res_m / res_m(first step) <= tol
    max_steps: int = 1000      # step cap
    fstore: str = "f64"


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    steps: int = 0
    converged: bool = False
    residual: float = float("nan")
    footprint: int = 0
    updates: int = 0           # cell-velocity updates performed
    W: Optional[np.ndarray] = None
    q: Optional[np.ndarray] = None
    error: str = ""

    @property
    def time_to_result(self) -> float:
        return self.finished - self.arrival


class GpuBackend:
    """Runs the admitted cases through the HIP library: all on one stream,
    advanced by batched steps (batched=True), or each on its own stream."""

    def __init__(self, batched: bool = True, max_cases: int = 64):
        import ctypes
        import torch
        from . import ugks
        if not torch.cuda.is_available():
            raise RuntimeError("GpuBackend needs the GPU")
        self._torch, self._ugks, self._ctypes = torch, ugks, ctypes
        self.batched = batched
        self._stream = torch.cuda.Stream()  # default priority
        self._batch = ugks.Batch(max_cases, ctypes.c_void_p(self._stream.cuda_stream)) if batched else None

    def footprint(self, req: Request) -> int:
        return self._ugks.footprint_estimate(req.case, req.fstore)

    def start(self, req: Request):
        stream = self._stream if self.batched else self._torch.cuda.Stream()
        s = self._ugks.Solver(req.case, fstore=req.fstore, stream=self._ctypes.c_void_p(stream.cuda_stream))
        s._serve_stream = stream            # keep the stream alive with the solver
        return s

    def step_batch(self, solvers, n: int):
        """n steps of every solver in batched launches (one per dimension)."""
        for dim in sorted({s.dim for s in solvers}):
            self._batch.step([s for s in solvers if s.dim == dim], n)


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 16, chunk: int = 10, backend=None,
                 clock: Callable[[], float] = time.perf_counter, idle: Callable[[], None] = lambda: time.sleep(1e-4)):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.backend = backend if backend is not None else GpuBackend()
        self.clock = clock
        self.idle = idle
        self.peak_used = 0
        self.log: List[tuple] = []   # (time, event, rid, bytes in use)

    def run(self, requests: List[Request]) -> List[Result]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results = {r.rid: Result(r.rid, r.arrival) for r in requests}
        batched = hasattr(self.backend, "step_batch") and getattr(self.backend, "batched", True)
        # rid -> [request, solver, footprint, first residual, steps queued, running]
        active = {}
        used = 0
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            progressed = False
            # admission: arrival order, while a slot is free and the footprint fits
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                req = pending[0]
                res = results[req.rid]
                fp = self.backend.footprint(req)
                res.footprint = fp
                if fp <= 0 or fp > self.budget:
                    pending.pop(0)
                    res.error = f"footprint {fp} B exceeds the budget of {self.budget} B"
                    res.finished = now
                    progressed = True
                    continue
                if used + fp > self.budget:
                    break
                pending.pop(0)
                try:
                    solver = self.backend.start(req)
                    if not batched:
                        solver.step_async(1)   # the first step's residual normalises the rest
                except Exception as exc:       # creation failure is reported, not fatal
                    res.error = str(exc)
                    res.finished = self.clock() - t0
                    progressed = True
                    continue
                used += fp
                self.peak_used = max(self.peak_used, used)
                res.admitted = now
                active[req.rid] = [req, solver, fp, None, 0 if batched else 1, not batched]
                self.log.append((now, "admit", req.rid, used))
                progressed = True
            # progress of the running cases
            for rid in list(active):
                req, solver, fp, r0, queued, running = active[rid]
                if not running:
                    continue
                res = results[rid]
                try:
                    r = solver.poll()
                except Exception as exc:
                    r, res.error = None, str(exc)
                if r is None and not res.error:
                    continue
                progressed = True
                active[rid][5] = False
                res.steps = queued
                done = bool(res.error)
                if not done:
                    if r0 is None:
                        r0 = np.where(r > 0, r, 1.0)
                        active[rid][3] = r0
                    res.residual = float(np.max(r / r0))
                    res.converged = res.residual <= req.tol
                    done = res.converged or queued >= req.max_steps
                if done:
                    if not res.error:
                        res.W, res.q = solver.macros()
                    res.updates = res.steps * solver.nc * solver.nv
                    solver.close()
                    del active[rid]
                    used -= fp
                    res.finished = self.clock() - t0
                    self.log.append((res.finished, "retire", rid, used))
                elif not batched:
                    n = min(self.chunk, req.max_steps - queued)
                    solver.step_async(n)
                    active[rid][4] = queued + n
                    active[rid][5] = True
            # batched: every case not running gets its next chunk, in one
            # batched step per chunk length (1 for a case's first step)
            if batched:
                groups = {}
                for rid, (req, solver, fp, r0, queued, running) in active.items():
                    if not running:
                        n = 1 if queued == 0 else min(self.chunk, req.max_steps - queued)
                        groups.setdefault(n, []).append(rid)
                for n, rids in sorted(groups.items()):
                    try:
                        self.backend.step_batch([active[rid][1] for rid in rids], n)
                    except Exception as exc:
                        for rid in rids:
                            results[rid].error = str(exc)
                            active[rid][5] = True     # retired by the next poll
                        continue
                    for rid in rids:
                        active[rid][4] += n
                        active[rid][5] = True
                    self.log.append((self.clock() - t0, "batch", tuple(rids), n))
                    progressed = True
            if not progressed:
                self.idle()
        return [results[r.rid] for r in requests]

    @staticmethod
    def summary(results: List[Result]) -> dict:
        """Time-to-converged percentiles over the cases that reached their
        tolerance; the cases stopped by the step cap are counted and timed
        apart (their time measures the cap, not convergence)."""
        ok = [r for r in results if not r.error]
        conv = [r for r in ok if r.converged]
        capped = [r for r in ok if not r.converged]

        def pct(rs, q):
            return float(np.percentile([r.time_to_result for r in rs], q)) if rs else float("nan")

        span = max((r.finished for r in ok), default=0.0) - min((r.arrival for r in ok), default=0.0)
        ups = sum(r.updates for r in ok)
        return {
            "cases": len(results),
            "completed": len(ok),
            "converged": len(conv),
            "capped": len(capped),
            "rejected_or_failed": len(results) - len(ok),
            "p50_time_to_converged_s": pct(conv, 50),
            "p99_time_to_converged_s": pct(conv, 99),
            "steps_to_converge_p50": float(np.percentile([r.steps for r in conv], 50)) if conv else float("nan"),
            "steps_to_converge_max": int(max((r.steps for r in conv), default=0)),
            "p50_time_to_result_capped_s": pct(capped, 50),
            "makespan_s": float(span),
            "updates_per_s": float(ups / span) if span > 0 else 0.0,
        }


def poisson_stream(n_cases: int = 128, rate: float = 4.0, seed: int = 0, n_cells=(2000, 50000), n_1d=(20, 64),
                   ma=(0.5, 6.0), kn=(1e-3, 1.0), tol: float = 1e-6, max_steps: int = 1000, fstore: str = "f32",
                   dv_max: float = 0.7, r_far: float = 15.0, h_first: float = 0.02, quad_rings: int = 0):
    """Requests of the serving workload: Poisson arrivals (rate per second),
    cylinder cases with N_c log-uniform in n_cells (all triangles), N_1D x N_1D
    velocity grids with N_1D uniform, Ma uniform, Kn log-uniform; velocity
    half-width max(6, 0.4 U_inf + 6 sqrt(R T_s)) around 0 (the paper's sizing
    rule for its cylinder velocity mesh, Section 4.1).  N_1D is raised where
    needed so that the spacing stays below dv_max (in units of the free-stream
    sqrt(2 R T)): a coarser grid cannot carry the free-stream Maxwellian."""
    import math
    from . import cases
    rng = cases.SplitMix64(seed)
    t = 0.0
    out = []
    for rid in range(n_cases):
        t += -math.log(1.0 - rng.uniform()) / rate
        nc_target = math.exp(math.log(n_cells[0]) + rng.uniform() * (math.log(n_cells[1]) - math.log(n_cells[0])))
        n1 = int(n_1d[0] + rng.uniform() * (n_1d[1] - n_1d[0] + 1))
        m = ma[0] + rng.uniform() * (ma[1] - ma[0])
        k = math.exp(math.log(kn[0]) + rng.uniform() * (math.log(kn[1]) - math.log(kn[0])))
        # all-triangle O-grid: n_theta x n_r quads, each cut in two
        n_r = max(4, int(round(math.sqrt(nc_target / 8.0))))
        n_theta = max(8, int(round(nc_target / (2 * n_r))))
        T_s = 1.0 + m * m / 3.0
        u_inf = m * cases.sound_speed(1.0)
        half = max(6.0, 0.4 * u_inf + 6.0 * math.sqrt(cases.R_GAS * T_s))
        n1 = max(n1, int(math.ceil(2.0 * half / dv_max)) + 1)    # trapezoid points: spacing 2 half / (n1 - 1)
        case = cases.case_cylinder(n_theta=n_theta, n_r=n_r, n_tri_rings=max(0, n_r - quad_rings), nv=n1,
                                   half_width=half, ma=m, kn=k, h_first=h_first, r_far=r_far, seed=seed + rid)
        case["name"] += f"_ma{m:.2f}_kn{k:.1e}"
        out.append(Request(rid, case, arrival=t, tol=tol, max_steps=max_steps, fstore=fstore))
    return out


def converging_stream(n_cases: int = 16, seed: int = 1, max_steps: int = 60000, tol: float = 1e-6):
    """A stream of small cases that reach a relative residual of 1e-6 within
    the step cap: supersonic cylinders (Ma 1.5-3, Kn 0.05-1) in a radius-5
    far field, 2k-5k cells (quadrilaterals in the six wall rings, triangles
    outside), 20^2-32^2 velocities, arriving at 8 per second.  f is kept in
    FP64: in FP32 the relative residual levels off near 2e-6, above the
    tolerance."""
    return poisson_stream(n_cases=n_cases, rate=8.0, seed=seed, n_cells=(2000, 5000), n_1d=(20, 32),
                          ma=(1.5, 3.0), kn=(0.05, 1.0), tol=tol, max_steps=max_steps, fstore="f64",
                          r_far=5.0, h_first=0.05, quad_rings=6)
