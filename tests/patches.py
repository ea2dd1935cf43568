"""Test helper: the neighbourhood of a few cells cut out of a mesh as a case
of its own.

One step of the scheme changes a cell from what lies within two faces of it:
its own limited slope and those of its face neighbours (which read their
neighbours' f), the interface states of its faces (the limited gradients of W
of the cell and its neighbours, which read their neighbours' W, and both
cells' heat flux) and the wall densities of its own wall faces.  Everything
else it needs is the global time step.  A patch made of the cells within two
faces of the chosen centres, run with the full mesh's time step, therefore
gives the centres the same step as the full mesh: the centres and their
neighbours keep every face they had, and only the outer ring's faces to cells
left out become far-field faces (which changes the outer ring's own update,
never the centres').  Faces keep their relative order, so every kept cell
sums over its faces in the same order as in the full mesh.

This lets the oracle check a mesh too large for it on sampled cells."""
import numpy as np

from paper_2412_06546_amd import cases


def rings(case, centres, n_rings=2):
    """The cells within n_rings faces of the centres (the centres first, then
    the rest in increasing index)."""
    fc = np.asarray(case["mesh"]["face_cells"])
    nc = len(case["mesh"]["cell_volume"])
    inner = fc[:, 1] >= 0
    a = np.concatenate([fc[inner, 0], fc[inner, 1]])
    b = np.concatenate([fc[inner, 1], fc[inner, 0]])
    order = np.argsort(a, kind="stable")
    a, b = a[order], b[order]
    start = np.searchsorted(a, np.arange(nc + 1))
    centres = [int(c) for c in centres]
    seen = set(centres)
    front = list(centres)
    for _ in range(n_rings):
        nxt = set()
        for c in front:
            nxt.update(int(x) for x in b[start[c]:start[c + 1]])
        nxt -= seen
        seen |= nxt
        front = sorted(nxt)
    rest = sorted(seen - set(centres))
    return np.array(list(dict.fromkeys(centres)) + rest, dtype=np.int64)


def patch_case(case, centres, dt, n_rings=2, cut_bc_id=0):
    """The cells within n_rings faces of the centres as a case of their own,
    stepped with the given time step.  Returns (patch, cells): the patch's
    cell p is the case's cell cells[p]; the centres come first, in the order
    given.  A face to a cell left out becomes an outflow far-field face of
    the kept cell (boundary row cut_bc_id), its normal turned out of that
    cell."""
    m = case["mesh"]
    cells = rings(case, centres, n_rings)
    nc = len(m["cell_volume"])
    local = np.full(nc, -1, dtype=np.int64)
    local[cells] = np.arange(len(cells))
    fc = np.asarray(m["face_cells"])
    lft = local[fc[:, 0]]
    rgt = np.where(fc[:, 1] >= 0, local[np.maximum(fc[:, 1], 0)], -1)
    keep = np.nonzero((lft >= 0) | (rgt >= 0))[0]          # original order
    l, r = lft[keep], rgt[keep]
    boundary = fc[keep, 1] < 0
    flip = (l < 0) & (r >= 0)                               # only the right cell kept
    cut = ~boundary & ((l < 0) | (r < 0))
    new_fc = np.stack([np.where(flip, r, l), np.where(cut | boundary, -1, r)], axis=1).astype(np.int32)
    nrm = np.asarray(m["face_normal"])[keep].copy()
    nrm[flip] *= -1.0
    bc = np.asarray(m["face_bc"])[keep].copy()
    bid = np.asarray(m["face_bc_id"])[keep].copy()
    bc[cut] = cases.BC_OUTFLOW
    bid[cut] = cut_bc_id
    fcen = np.asarray(m["face_centroid"])[keep].copy()
    mesh = dict(m)
    if m.get("face_shift") is not None:
        # a face centroid is given in the left cell's frame: a periodic face
        # whose right cell is kept alone moves into that cell's frame
        shift = np.asarray(m["face_shift"])[keep].copy()
        fcen[flip] -= shift[flip]
        shift[cut] = 0.0
        mesh["face_shift"] = shift
    mesh.update(cell_volume=np.asarray(m["cell_volume"])[cells], cell_centroid=np.asarray(m["cell_centroid"])[cells],
                face_cells=new_fc, face_normal=nrm, face_area=np.asarray(m["face_area"])[keep],
                face_centroid=fcen, face_bc=bc.astype(np.int32), face_bc_id=bid.astype(np.int32))
    gas = dict(case["gas"])
    gas["dt_override"] = float(dt)
    patch = dict(case)
    patch.update(name=case["name"] + f"_patch{len(cells)}", mesh=mesh, gas=gas,
                 prim0=np.asarray(case["prim0"])[cells])
    return patch, cells
