"""Two-stage update (Section 3.2) against the basic algorithm (Section 3.1).

The oracle updates f velocity by velocity in place with the split of
Eqs. microS1/microS2 and evolves the wall flux after the velocity loop, as in
Algorithm 1.  oracle/brute.py is an independent implementation that stores
every gradient and residual and applies the one-shot implicit update of
Eq. microscopicUpdata.  The algebra says they are the same scheme; here they
must agree to round-off on tiny meshes with every kind of face.
"""
import numpy as np
import pytest

import oracle
from oracle.brute import BruteUGKS
from paper_2412_06546_amd import cases


def _tiny_cases():
    out = []
    m = cases.periodic_triangles(3, 3, 1.5, 1.0, seed=4)
    nc = len(m["cell_volume"])
    x = m["cell_centroid"]
    p0 = np.stack([1 + 0.2 * np.sin(2 * np.pi * x[:, 0] / 1.5), 0.1 * np.cos(2 * np.pi * x[:, 1]),
                   np.full(nc, -0.05), 1 + 0.1 * np.cos(2 * np.pi * x[:, 0] / 1.5)], 1)
    out.append(("periodic triangles", dict(mesh=m, vgrid=cases.tensor_vgrid(6, 4.0, 2),
                                           gas=cases.gas_params(2 / 3, 0.81, 0.05), prim0=p0)))
    m = cases.channel_quads(3, 3, 1.0, 1.0, y_bc=(cases.BC_WALL, 1))
    nc = len(m["cell_volume"])
    x = m["cell_centroid"]
    p0 = np.stack([1 + 0.1 * x[:, 1], 0.3 * np.ones(nc), 0.05 * np.sin(2 * np.pi * x[:, 0]), 1 + 0.2 * x[:, 0]], 1)
    bc = np.array([[1.0, 0.0, 0.0, 1.0], [1.0, 0.2, 0.0, 1.3]])
    out.append(("channel between walls", dict(mesh=m, vgrid=cases.tensor_vgrid(7, 4.0, 2),
                                              gas=cases.gas_params(2 / 3, 0.81, 0.08, bc_prim=bc), prim0=p0)))
    c = cases.case_cylinder(n_theta=12, n_r=3, n_tri_rings=1, nv=12, half_width=8.0, h_first=0.05, r_far=3.0,
                            ma=2.0)
    out.append(("cylinder: wall, inflow, outflow", c))
    c = cases.case_box_wave_3d(n=3, kind="tet", nv=4, half_width=3.0)
    out.append(("3D tetrahedra", c))
    c = cases.case_channel_3d(n=3, kind="prism", nv=4, half_width=3.0)
    out.append(("3D prisms between walls", c))
    return out


@pytest.mark.parametrize("name,case", _tiny_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_two_stage_equals_one_shot(name, case):
    o = oracle.Oracle(case)
    b = BruteUGKS(case)
    assert o.dt == pytest.approx(b.dt, rel=1e-14)
    for _ in range(3):
        o.step(1)
        b.step()
    W, q = o.macros()
    f = o.f()
    np.testing.assert_allclose(b.W, W, rtol=1e-13, atol=1e-14 * np.abs(W).max())
    np.testing.assert_allclose(b.q, q, rtol=1e-11, atol=1e-13 * max(np.abs(q).max(), 1e-3))
    np.testing.assert_allclose(b.f, f, rtol=1e-12, atol=1e-14 * np.abs(f).max())
    assert np.abs(W - o.macros()[0]).max() == 0.0
