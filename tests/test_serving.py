"""Scheduling logic of the serving loop, on a fake backend (no GPU)."""
import numpy as np
import pytest

from paper_2412_06546_amd.serve import Request, Server


class FakeJob:
    def __init__(self, clock, cost, decay):
        self.clock, self.cost, self.decay = clock, cost, decay
        self.nc, self.nv = 10, 4
        self.busy_until = None
        self.done_steps = 0
        self.r = 1.0

    def step_async(self, n):
        assert self.busy_until is None, "one batch outstanding at a time"
        self.busy_until = self.clock.t + self.cost * n
        self.n = n

    def poll(self):
        if self.busy_until is None or self.clock.t < self.busy_until:
            return None
        self.busy_until = None
        self.done_steps += self.n
        self.r = self.decay ** (self.done_steps - 1)
        return np.array([self.r, 1.0 * self.r, 0.5 * self.r, 2.0 * self.r])

    def macros(self):
        return np.full((self.nc, 4), float(self.done_steps)), np.zeros((self.nc, 2))

    def close(self):
        self.closed = True


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 0.01


class FakeBackend:
    def __init__(self, clock, sizes, costs, decays):
        self.clock, self.sizes, self.costs, self.decays = clock, sizes, costs, decays
        self.started = []

    def footprint(self, req):
        return self.sizes[req.rid]

    def start(self, req):
        self.started.append(req.rid)
        return FakeJob(self.clock, self.costs[req.rid], self.decays[req.rid])


def _run(sizes, costs, decays, arrivals, budget, max_active=8, tol=1e-3, max_steps=200, chunk=5):
    clock = FakeClock()
    be = FakeBackend(clock, sizes, costs, decays)
    srv = Server(budget, max_active=max_active, chunk=chunk, backend=be, clock=clock, idle=clock.tick)
    reqs = [Request(i, {}, arrival=a, tol=tol, max_steps=max_steps) for i, a in enumerate(arrivals)]
    return srv, be, srv.run(reqs)


def test_admission_respects_budget_and_order():
    sizes = [40, 30, 50, 20, 60, 10]
    srv, be, res = _run(sizes, [0.02] * 6, [0.5] * 6, [0.0, 0.0, 0.01, 0.02, 0.02, 0.5], budget=100)
    assert srv.peak_used <= 100
    assert be.started == sorted(be.started)          # arrival (FIFO) order
    assert all(r.error == "" for r in res)
    # memory in use never exceeds the budget at any logged instant
    assert max(u for _, _, _, u in srv.log) <= 100
    # requests waited for memory: some were admitted after they arrived
    assert any(r.admitted > r.arrival + 1e-9 for r in res)


def test_oversized_request_is_rejected_without_blocking_the_queue():
    srv, be, res = _run([50, 500, 20], [0.01] * 3, [0.5] * 3, [0.0, 0.0, 0.0], budget=100)
    assert "exceeds the budget" in res[1].error
    assert res[0].error == "" and res[2].error == ""
    assert 1 not in be.started


def test_convergence_and_step_cap():
    # decay 0.5 per step reaches 1e-3 after 11 steps; decay 0.999 never does
    srv, be, res = _run([10, 10], [0.01, 0.01], [0.5, 0.999], [0.0, 0.0], budget=100, tol=1e-3, max_steps=50)
    assert res[0].converged and res[0].steps < 50 and res[0].residual <= 1e-3
    assert not res[1].converged and res[1].steps == 50
    s = Server.summary(res)
    assert s["converged"] == 1 and s["capped"] == 1
    # time-to-converged counts the converged case only; the capped one is apart
    assert s["p50_time_to_converged_s"] == pytest.approx(res[0].time_to_result)
    assert s["p99_time_to_converged_s"] == pytest.approx(res[0].time_to_result)
    assert s["p50_time_to_result_capped_s"] == pytest.approx(res[1].time_to_result)
    assert s["steps_to_converge_max"] == res[0].steps
    # none converged: the percentiles are not numbers, the capped count is all
    s2 = Server.summary([res[1]])
    assert s2["converged"] == 0 and s2["capped"] == 1 and s2["p50_time_to_converged_s"] != s2["p50_time_to_converged_s"]


def test_slots_limit_concurrency():
    srv, be, res = _run([1] * 6, [0.05] * 6, [0.9] * 6, [0.0] * 6, budget=100, max_active=2, max_steps=20)
    live = 0
    peak = 0
    for _, ev, _, _ in srv.log:
        live += 1 if ev == "admit" else -1
        peak = max(peak, live)
    assert peak == 2
    assert all(r.steps == 20 for r in res)


def test_poisson_stream_recipe():
    """Arrivals increase, every velocity grid resolves the free stream (spacing
    at most dv_max), meshes stay within the requested cell range."""
    from paper_2412_06546_amd.serve import poisson_stream
    reqs = poisson_stream(n_cases=4, n_cells=(2000, 3000), n_1d=(20, 24), ma=(5.5, 6.0), max_steps=7)
    arr = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    for r in reqs:
        u = r.case["vgrid"]["u"]
        n1 = int(round(np.sqrt(len(u))))
        du = np.diff(np.unique(u[:, 0])).max()
        assert du <= 0.7 + 1e-12 and n1 > 24
        assert 1500 <= len(r.case["mesh"]["cell_volume"]) <= 3500
        assert r.max_steps == 7 and "_ma" in r.case["name"]


class FakeBatchBackend(FakeBackend):
    """A backend with batched steps: every call advances several jobs."""

    def __init__(self, *a):
        super().__init__(*a)
        self.calls = []

    def step_batch(self, jobs, n):
        self.calls.append((len(jobs), n))
        for j in jobs:
            j.step_async(n)


def test_batched_rounds_respect_budget_and_step_counts():
    clock = FakeClock()
    n = 8
    sizes = [30, 40, 25, 60, 35, 20, 45, 50]
    be = FakeBatchBackend(clock, sizes, [0.01] * n, [0.5, 0.6, 0.7, 0.8, 0.5, 0.9, 0.6, 0.95])
    reqs = [Request(i, None, arrival=0.01 * i, tol=1e-3, max_steps=40) for i in range(n)]
    srv = Server(120, max_active=4, chunk=5, backend=be, clock=clock, idle=clock.tick)
    res = srv.run(reqs)
    assert all(not r.error for r in res)
    assert srv.peak_used <= 120
    assert max(k for k, _ in be.calls) > 1                      # several cases per batched step
    assert all(nn == 1 or nn <= 5 for _, nn in be.calls)          # a first single step, then chunks
    for r, d in zip(res, [0.5, 0.6, 0.7, 0.8, 0.5, 0.9, 0.6, 0.95]):
        assert r.steps <= 40
        assert r.converged == (d ** (r.steps - 1) <= 1e-3)
        if not r.converged:
            assert r.steps == 40
    admitted = sorted(res, key=lambda r: r.admitted)
    assert [r.rid for r in admitted] == sorted(r.rid for r in res)  # arrival order
