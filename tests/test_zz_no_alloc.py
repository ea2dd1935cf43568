"""ugks_batch_step_static (no allocation: a fixed device array holds the
batch descriptors) against ugks_batch_step, the entry point it is a variant
of: the same kernels, so the results must be bitwise equal.  Two calls in a
row, the second with fewer and smaller cases, so that the fixed array holds
the previous call's (larger) contents when it is reused."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2412_06546_amd import cases

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_06546_amd import ugks
    ugks.load_library()
    return ugks, torch


def _wait(solvers):
    out = []
    for s in solvers:
        r = None
        while r is None:
            r = s.poll()
        out.append(r)
    return out


def _state(s):
    W, q = s.macros()
    return W, q, s.f()


def test_static_batch_matches_the_batch_object():
    ugks, torch = _gpu()
    stream = torch.cuda.Stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    big = [cases.case_cylinder_small(), cases.case_periodic_wave(),
           cases.case_cylinder_small(n_theta=24, n_r=8, nv=20)]
    small = [cases.case_periodic_wave(nx=6, ny=4, nv=10)]
    stores = ["f64", "f32", "bf16"]
    print("static batch: 3 cases x 4 steps, then 1 case x 3 steps", flush=True)
    batch = ugks.Batch(4, h)
    for group, nsteps in ((big, 4), (small, 3)):
        ref = [ugks.Solver(c, fstore=stores[i % 3], stream=h) for i, c in enumerate(group)]
        got = [ugks.Solver(c, fstore=stores[i % 3], stream=h) for i, c in enumerate(group)]
        batch.step(ref, nsteps)
        rr = _wait(ref)
        ugks.batch_step_static(got, nsteps, h)
        rg = _wait(got)
        for a, b, ra, rb in zip(ref, got, rr, rg):
            assert a.step_count == b.step_count == nsteps
            assert np.array_equal(ra, rb)
            for x, y in zip(_state(a), _state(b)):
                assert np.array_equal(x, y)
        for s in ref + got:
            s.close()


def test_static_batch_rejects_too_many_cases():
    ugks, torch = _gpu()
    stream = torch.cuda.Stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    s = ugks.Solver(cases.case_periodic_wave(nx=6, ny=4, nv=6), stream=h)
    with pytest.raises(ugks.UgksError) as e:
        ugks.batch_step_static([s] * (ugks.UGKS_STATIC_BATCH_MAX + 1), 1, h)
    assert e.value.code == ugks.UGKS_ERR_ARG and "64" in str(e.value)
    # one handle twice is refused too; the handle is untouched and steps on
    with pytest.raises(ugks.UgksError):
        ugks.batch_step_static([s, s], 1, h)
    ugks.batch_step_static([s], 2, h)
    _wait([s])
    assert s.step_count == 2
