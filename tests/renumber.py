"""Test helper: the same case with its cells and faces renumbered."""
import numpy as np


def renumber(case, seed):
    """The same case with cells and faces renumbered by seeded permutations;
    returns the case and new -> old cell map."""
    rng = np.random.default_rng(seed)
    m = dict(case["mesh"])
    nc, nf = len(m["cell_volume"]), len(m["face_area"])
    cp, fp = rng.permutation(nc), rng.permutation(nf)      # new index -> old index
    inv = np.empty(nc, dtype=np.int64)
    inv[cp] = np.arange(nc)
    m["cell_volume"], m["cell_centroid"] = m["cell_volume"][cp], m["cell_centroid"][cp]
    fc = m["face_cells"][fp].copy()
    fc[:, 0] = inv[fc[:, 0]]
    fc[fc[:, 1] >= 0, 1] = inv[fc[fc[:, 1] >= 0, 1]]
    m["face_cells"] = fc
    for k in ("face_normal", "face_area", "face_centroid", "face_bc", "face_bc_id"):
        m[k] = m[k][fp]
    if m.get("face_shift") is not None:
        m["face_shift"] = m["face_shift"][fp]
    out = dict(case)
    out["mesh"], out["prim0"] = m, case["prim0"][cp]
    out["name"] = case["name"] + "_renumbered"
    return out, cp
