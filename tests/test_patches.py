"""The patch method that checks the full-size lifting body on sampled cells
(tests/patches.py), pinned on meshes the oracle runs whole: one oracle step
on the cells within two faces of a few centres, with the full mesh's time
step, gives the centres exactly the full mesh's step (W, q and f, bit for
bit), while one ring is not enough (the centres then differ) and the outer
ring itself does differ (the cut is real).  Cases: the cylinder cut-down
(wall, far field, quadrilaterals and triangles), a hexahedral sphere shell,
a periodic box of tetrahedra (periodic faces cut), a small lifting body
(hexahedra and prisms, octree velocity set)."""
import numpy as np
import pytest

import oracle
from paper_2412_06546_amd import cases
from patches import patch_case

CASES = {
    "cylinder": lambda: cases.case_cylinder_small(),
    "sphere_hex": lambda: cases.case_sphere(n=4, n_r=8, nv=8, half_width=8.0, kind="hex"),
    "box_tet": lambda: cases.case_box_wave_3d(n=4, kind="tet", nv=6),
    "lifting_body": lambda: cases.case_lifting_body(n=4, n_r=8, n_prism_columns=4, n_vel=300),
}


def _centres(c):
    """A wall cell, a far-field cell, a middle and the last cell."""
    nc = len(c["mesh"]["cell_volume"])
    fb = np.asarray(c["mesh"]["face_bc"])
    fcl = np.asarray(c["mesh"]["face_cells"])
    wall = fcl[fb == cases.BC_WALL, 0]
    far = fcl[(fb == cases.BC_INFLOW) | (fb == cases.BC_OUTFLOW), 0]
    cen = [int(wall[0]) if len(wall) else 0, int(far[len(far) // 2]) if len(far) else 1, nc // 2, nc - 1]
    return list(dict.fromkeys(cen))


@pytest.mark.parametrize("which", sorted(CASES))
def test_two_ring_patch_reproduces_the_full_step(which):
    c = CASES[which]()
    o = oracle.Oracle(c)
    o.step(1)
    W, q = o.macros()
    f = o.f()
    cen = _centres(c)
    k = len(cen)
    diffs = {}
    for n_rings in (1, 2):
        p, cells = patch_case(c, cen, o.dt, n_rings=n_rings)
        assert list(cells[:k]) == cen and len(cells) < len(W)
        op = oracle.Oracle(p)
        assert op.dt == o.dt
        op.step(1)
        Wp, qp = op.macros()
        fp = op.f()
        diffs[n_rings] = max(np.abs(Wp[:k] - W[cen]).max(), np.abs(qp[:k] - q[cen]).max(),
                             np.abs(fp[:k] - f[cen]).max())
        if n_rings == 2:
            assert np.abs(Wp[k:] - W[cells[k:]]).max() > 1e-6    # the outer ring is cut
    assert diffs[2] == 0.0, diffs
    assert diffs[1] > 1e-8, diffs
