"""Serving on the GPU: admission by footprint, overlapped cases, and each
result equal to the same case run alone (and to the oracle)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_06546_amd import cases

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_06546_amd import ugks
    ugks.load_library()
    return ugks


def _mix():
    return [
        cases.case_periodic_wave(nx=10, ny=6, nv=20, seed=1),
        cases.case_cylinder_small(n_theta=32, n_r=10, nv=20),
        cases.case_periodic_wave(nx=16, ny=8, nv=32, seed=2, Pr=2.0 / 3.0, omega=0.81),
        cases.case_box_wave_3d(n=3, kind="prism", nv=8),
        cases.case_cylinder_small(n_theta=40, n_r=12, nv=28, ma=3.0),
        cases.case_periodic_wave(nx=8, ny=8, nv=16, seed=3),
    ]


def test_footprint_estimate_matches_allocation():
    ugks = _gpu()
    cs = _mix()
    c = cases.case_cylinder_small()
    keep = (c["vgrid"]["u"] ** 2).sum(1) < 100
    c["vgrid"] = dict(dim=2, u=np.ascontiguousarray(c["vgrid"]["u"][keep]), w=np.ascontiguousarray(c["vgrid"]["w"][keep]))
    cs.append(c)
    for c in cs:
        dim = c["mesh"]["dim"]
        for fs in ("f64", "f32", "bf16"):
            for sw in ("auto", "gather", "push"):
                est = ugks.footprint_estimate(c, fs, sweep=sw)
                s = ugks.Solver(c, fstore=fs, sweep=sw)
                assert s.footprint_bytes == est, (c.get("name"), fs, sw)
                # the automatic choice: push, except 2D FP64 and BF16 f
                auto = "gather" if fs == "bf16" or (dim == 2 and fs == "f64") else "push"
                assert s.sweep == (auto if sw == "auto" else sw), (c.get("name"), fs, sw)
                assert (s.n_colours > 0) == (s.sweep == "push")
                s.close()
    # BF16 f pushes in place too (an FP32 ring)
    s = ugks.Solver(cs[0], fstore="bf16", mem="in-place", sweep="push")
    assert s.sweep == "push"
    assert s.footprint_bytes == ugks.footprint_estimate(cs[0], "bf16", "in-place", sweep="push")
    s.close()


@pytest.mark.parametrize("batched", [True, False])
def test_each_result_in_the_mix_equals_the_result_alone(batched):
    ugks = _gpu()
    from paper_2412_06546_amd.serve import GpuBackend, Request, Server
    cs = _mix()
    steps = 25
    fps = [ugks.footprint_estimate(c) for c in cs]
    budget = sorted(fps)[-1] + sorted(fps)[-2]           # at most about two at a time
    reqs = [Request(i, c, arrival=0.002 * i, tol=0.0, max_steps=steps) for i, c in enumerate(cs)]
    print(f"serving {len(cs)} cases, budget {budget} B", flush=True)
    srv = Server(budget, max_active=4, chunk=7, backend=GpuBackend(batched=batched))
    res = srv.run(reqs)
    s = Server.summary(res)
    print(s, flush=True)
    assert s["completed"] == len(cs)
    assert srv.peak_used <= budget
    assert any(r.admitted > r.arrival for r in res)      # some waited for memory
    for r, c in zip(res, cs):
        assert r.steps == steps
        # batched rounds run the gather sweep (ugks_batch_step), a stream per
        # case the default (push) sweep: the lone run takes the same one
        alone = ugks.Solver(c, sweep="gather" if batched else "auto")
        alone.step(steps)
        W, q = alone.macros()
        alone.close()
        assert np.array_equal(r.W, W), r.rid
        assert np.array_equal(r.q, q), r.rid
        # and the served result against the oracle
        o = oracle.Oracle(c)
        o.step(steps)
        Wo, _ = o.macros()
        scale = np.abs(Wo).max(axis=0)
        scale[1:-1] = np.maximum(scale[1:-1], Wo[:, 0].max())
        assert (np.abs(r.W - Wo).max(axis=0) / scale).max() <= 1e-12, r.rid


def test_async_steps_match_synchronous_steps():
    ugks = _gpu()
    c = cases.case_cylinder_small()
    a, b = ugks.Solver(c), ugks.Solver(c)
    a.step(12)
    b.step_async(5)
    while b.poll() is None:
        pass
    b.step_async(7)
    r = None
    while r is None:
        r = b.poll()
    assert np.array_equal(a.macros()[0], b.macros()[0])
    with pytest.raises(ugks.UgksError):
        b.step_async(1)
        b.step_async(1)    # a second batch before the first was polled


def _scattered(c, seed):
    u, w = c["vgrid"]["u"], c["vgrid"]["w"]
    rng = np.random.default_rng(seed)
    c["vgrid"] = dict(dim=c["mesh"]["dim"], u=np.ascontiguousarray(u + rng.uniform(-1e-3, 1e-3, u.shape)),
                      w=np.ascontiguousarray(w))
    return c


def test_batched_steps_are_bitwise_those_of_each_case_alone():
    """Cases of different sizes, velocity sets (Cartesian tables, scattered
    points), storage precisions and stage-1 placement (LDS or f_out) stepped
    together by ugks_batch_step, twice, against each stepped alone."""
    import ctypes
    import torch
    ugks = _gpu()
    mix = [(cases.case_periodic_wave(nx=10, ny=6, nv=20, seed=1), "f64"),
           (cases.case_cylinder_small(n_theta=32, n_r=10, nv=60), "f64"),     # slab too big for LDS
           (cases.case_cylinder_small(n_theta=24, n_r=8, nv=24), "f32"),
           (_scattered(cases.case_periodic_wave(nx=6, ny=6, nv=26, seed=4), 9), "f64"),     # too many axis values for tables
           (cases.case_periodic_wave(nx=12, ny=4, nv=16, seed=5), "bf16")]
    stream = torch.cuda.Stream()
    sh = ctypes.c_void_p(stream.cuda_stream)
    batch = ugks.Batch(8, sh)
    solvers = [ugks.Solver(c, fstore=fs, stream=sh) for c, fs in mix]
    assert not solvers[3].tensor_grid and solvers[0].tensor_grid
    print(f"batch of {len(solvers)} cases", flush=True)
    for n in (3, 4):
        batch.step(solvers, n)
        for s in solvers:
            r = None
            while r is None:
                r = s.poll()
    for (c, fs), s in zip(mix, solvers):
        alone = ugks.Solver(c, fstore=fs, sweep="gather")   # the batched kernels gather
        alone.step(7)
        Wa, qa = alone.macros()
        Wb, qb = s.macros()
        assert np.array_equal(Wa, Wb) and np.array_equal(qa, qb), c["name"]
        assert np.array_equal(alone.f(), s.f()), c["name"]
        assert s.step_count == 7
        alone.close()
    with pytest.raises(ugks.UgksError):
        batch.step([solvers[0], ugks.Solver(mix[0][0])], 1)       # not on the batch's stream
    for s in solvers:
        s.close()
    batch.close()
