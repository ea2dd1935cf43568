"""Pins of the oracle's steady-state residual and of the first-order fallback
of its macroscopic reconstruction.

The residual reported after a step is, per conservative component, the L2
norm over cells of W^{n+1} - W^n (the convergence measure of a run to steady
state).  Here it is recomputed by definition from two reads of W around one
step.

The macroscopic reconstruction (Algorithm 1) drops a cell's gradient of W
to zero when its limited reconstruction at one of its face centroids has
rho <= 0 or a non-positive internal energy.  A cold gas with a strong
velocity wave triggers it: the limiter bounds each conservative component
separately, so the kinetic energy of a reconstructed face state can exceed
its total energy.  The test predicts the flagged cells with the independent
brute-force reconstruction (oracle/brute.py) and its own face-state check,
and then compares the oracle's step with the brute-force step there.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.brute import BruteUGKS
from paper_2412_06546_amd import cases
from special_cases import fallback_case


def _l2_change(W0, W1):
    return np.sqrt(((W1 - W0) ** 2).sum(0))


def _check_residual(o, nsteps):
    for _ in range(nsteps):
        W0, _ = o.macros()
        o.step(1)
        W1, _ = o.macros()
        got = o.residual()
        ref = _l2_change(W0, W1)
        # W1 - W0 differs from the step's increment by the rounding of W1
        # (at most one unit in the last place of each value)
        tol = 1e-14 * ref + 4e-16 * math.sqrt(len(W0)) * np.abs(W1).max(0)
        assert np.all(np.abs(got - ref) <= tol), (got, ref)
        assert np.all(ref > 0)


def test_residual_is_the_l2_change_of_W_periodic_wave():
    _check_residual(oracle.Oracle(cases.case_periodic_wave()), 3)


def test_residual_is_the_l2_change_of_W_cylinder_cut_down():
    c = cases.case_cylinder(n_theta=24, n_r=8, n_tri_rings=2, nv=16, half_width=12.0, h_first=0.02, r_far=6.0)
    _check_residual(oracle.Oracle(c), 2)


def test_residual_vanishes_for_a_uniform_state():
    mesh = cases.periodic_triangles(6, 4, 1.5, 1.0, seed=5)
    nc = len(mesh["cell_volume"])
    vg = cases.tensor_vgrid(12, 5.0, 2)
    gas = cases.gas_params(2 / 3, 0.81, cases.vhs_mu_ref(0.1, 0.81, 1.0), dim=2)
    o = oracle.Oracle(dict(mesh=mesh, vgrid=vg, gas=gas, prim0=np.tile([1.3, 0.4, -0.25, 1.2], (nc, 1))))
    W0, _ = o.macros()
    o.step(1)
    W1, _ = o.macros()
    # a uniform state does not change: the face fluxes cancel to round-off
    r = o.residual()
    assert np.all(r <= 1e-15 * math.sqrt(nc) * np.abs(W0).max(0))
    assert np.all(np.abs(r - _l2_change(W0, W1)) <= 4e-16 * math.sqrt(nc) * np.abs(W1).max(0))


def _predicted_fallback(b):
    """Cells whose limited reconstruction of W (brute force) is not physical
    at one of their face centroids, and the brute-force gradients."""
    nc, D = len(b.vol), b.D
    flags = np.zeros(nc, bool)
    grads = np.zeros((nc, D + 2, D))
    for i in range(nc):
        g = b.limited_grad(i, b.W)
        grads[i] = g
        for _, _, r in b.cell_faces[i]:
            Wf = b.W[i] + g @ r
            rho, mom, E = Wf[0], Wf[1:1 + D], Wf[-1]
            if not (rho > 0 and E - 0.5 * (mom @ mom) / rho > 0):
                flags[i] = True
    return flags, grads


def test_macro_fallback_fires_and_matches_brute_force():
    case = fallback_case()
    o = oracle.Oracle(case)
    b = BruteUGKS(case)
    for step in range(3):
        flags, grads = _predicted_fallback(b)
        if step == 0:
            assert 0 < flags.sum() < len(flags) // 2
        g, bad = o.macro_gradients()
        np.testing.assert_array_equal(bad, flags)
        assert np.all(g[bad] == 0.0)
        scale = np.abs(grads).max()
        np.testing.assert_allclose(g[~bad], grads[~bad], rtol=1e-12, atol=1e-13 * scale)
        # the cells that did not fall back carry a real gradient
        assert np.abs(g[~bad]).max() > 1e-3
        o.step(1)
        b.step()
        W, q = o.macros()
        np.testing.assert_allclose(b.W, W, rtol=1e-13, atol=1e-14 * np.abs(W).max())
        np.testing.assert_allclose(b.f, o.f(), rtol=1e-12, atol=1e-14 * np.abs(b.f).max())
