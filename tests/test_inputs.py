"""The synthetic inputs both implementations consume (paper_2412_06546_amd.cases):
every mesh is a set of closed, consistently oriented finite volumes, and every
velocity set integrates the Maxwellian it is meant to resolve.  Host only."""
import math

import numpy as np
import pytest

from paper_2412_06546_amd import cases


def _meshes():
    yield "periodic triangles", cases.periodic_triangles(6, 4, 1.5, 1.0, seed=3)
    yield "periodic quads", cases.periodic_quads(5, 3, 1.0, 0.6)
    yield "channel quads", cases.channel_quads(4, 5, 1.0, 1.0)
    yield "cylinder (cut-down)", cases.case_cylinder_small()["mesh"]
    for kind in ("hex", "tet", "prism"):
        yield f"3D periodic box ({kind})", cases.box_mesh_3d(3, 3, 3, kind=kind)
        yield f"3D channel ({kind})", cases.case_channel_3d(n=3, kind=kind)["mesh"]
    yield "sphere shell (tetrahedra)", cases.case_sphere(n=4, n_r=4, nv=4)["mesh"]
    # curved shells: their hexahedra have non-planar (bilinear) quadrilateral
    # faces, for which one centroid per face gives the volume only to a few
    # per cent on these coarse versions
    yield "sphere shell (hexahedra)", cases.case_sphere(n=4, n_r=4, nv=4, kind="hex")["mesh"]
    yield "lifting-body shell (hexahedra and prisms)", cases.case_lifting_body(
        n=6, n_r=8, n_prism_columns=10, n_base=6, n_vel=None)["mesh"]


@pytest.mark.parametrize("name,mesh", list(_meshes()), ids=lambda x: x if isinstance(x, str) else "")
def test_mesh_cells_are_closed_and_consistently_oriented(name, mesh):
    D = int(mesh["dim"])
    fc = np.asarray(mesh["face_cells"])
    n, S, xf = mesh["face_normal"], mesh["face_area"], mesh["face_centroid"]
    xc, vol = mesh["cell_centroid"], mesh["cell_volume"]
    shift = mesh.get("face_shift")
    shift = np.zeros_like(xf) if shift is None else shift
    nc = len(vol)
    inner = fc[:, 1] >= 0
    assert np.all(vol > 0) and np.all(S > 0)
    assert np.allclose((n ** 2).sum(1), 1.0, atol=1e-12)
    # closed: the outward area vectors of every cell sum to zero
    acc = np.zeros((nc, D))
    np.add.at(acc, fc[:, 0], S[:, None] * n)
    np.add.at(acc, fc[inner, 1], -S[inner, None] * n[inner])
    assert np.abs(acc).max() <= 1e-12 * S.max()
    # volumes by the divergence theorem, |Omega| = (1/D) sum S n . x_f (the
    # right cell sees its periodic image of the face)
    v = np.zeros(nc)
    np.add.at(v, fc[:, 0], S * (n * xf).sum(1) / D)
    np.add.at(v, fc[inner, 1], -S[inner] * (n[inner] * (xf[inner] - shift[inner])).sum(1) / D)
    assert np.allclose(v, vol, rtol=5e-2 if "shell (hexahedra" in name else 1e-9)
    # normals point from the left cell to the right one, and out of the domain
    d = xc[fc[inner, 1]] + shift[inner] - xc[fc[inner, 0]]
    assert np.all((d * n[inner]).sum(1) > 0)
    db = xf[~inner] - xc[fc[~inner, 0]]
    assert np.all((db * n[~inner]).sum(1) > 0)
    # boundary types match the face's cells
    assert np.all((np.asarray(mesh["face_bc"]) == 0) == inner)


@pytest.mark.parametrize("dim", [2, 3])
def test_cartesian_velocity_grid_integrates_the_maxwellian(dim):
    """Trapezoid weights on [-L, L]^dim: the moments 1, u, |u|^2 of a Maxwellian
    well inside the grid are those of the continuous one (the trapezoid rule
    converges spectrally for it)."""
    vg = cases.tensor_vgrid(32 if dim == 2 else 26, 7.0, dim)
    u, w = vg["u"], vg["w"]
    U = np.array([0.4, -0.3, 0.2][:dim])
    T = 1.3
    g = (1.0 / (math.pi * T)) ** (dim / 2) * np.exp(-((u - U) ** 2).sum(1) / T)
    assert (w * g).sum() == pytest.approx(1.0, abs=1e-10)
    assert np.allclose((w[:, None] * u * g[:, None]).sum(0), U, atol=1e-10)
    assert (w * (u ** 2).sum(1) * g).sum() == pytest.approx((U ** 2).sum() + dim * T / 2, rel=1e-10)
    assert w.sum() == pytest.approx(14.0 ** dim, rel=1e-12)


def test_octree_velocity_set_is_a_partition():
    """The unstructured (octree) set: its weights are the volumes of disjoint
    cells covering the box, so they sum to its volume before trimming, and
    every point lies in the box."""
    L = 15.0
    vg = cases.octree_vgrid(6, L, [([np.array([4.0, 0.0, 1.0]), np.zeros(3)], 6.5),
                                   ([np.array([4.0, 0.0, 1.0])], 2.2)])
    u, w = vg["u"], vg["w"]
    assert w.sum() == pytest.approx((2 * L) ** 3, rel=1e-12)
    assert np.all(np.abs(u) < L)
    assert len(np.unique(np.round(u, 12), axis=0)) == len(u)
