"""Seeded synthetic inputs for the UGKS step: meshes, velocity grids, gas data.

This module only builds inputs.  It holds none of the scheme's arithmetic
(no equilibria, fluxes, reconstructions or updates); both the HIP library and
the CPU oracle consume what it returns.  Every random choice is drawn from a
splitmix64 stream with an explicit seed.

Units follow the usual kinetic non-dimensionalisation: gas constant R = 1/2,
free-stream density and temperature 1, so the most probable speed
sqrt(2 R T) is 1 and lambda = 1/(2 R T) = 1/T.

A case is a plain dict:

  mesh   : dim, cell_volume[nc], cell_centroid[nc,dim], face_cells[nf,2]
           (right = -1 on a boundary), face_normal[nf,dim] (unit, left->right,
           outward on a boundary), face_area[nf], face_centroid[nf,dim]
           (in the left cell's frame), face_shift[nf,dim] (added to the right
           cell's centroid to place its periodic image next to the left cell),
           face_bc[nf] (0 interior/periodic, 1 inflow, 2 outflow, 3 wall),
           face_bc_id[nf] (row of gas['bc_prim']).
  vgrid  : dim, u[nv,dim], w[nv]   (velocity points and quadrature weights,
           Section 2.3: the integral over velocity space is sum_k Q_k V_k).
  gas    : Pr, omega, mu_ref, cfl, dt_override, limiter (0 none, 1
           Venkatakrishnan), limiter_k, bc_prim[nbc, dim+2] (rho, U, T).
  prim0  : [nc, dim+2] initial (rho, U, T) per cell.
"""
from __future__ import annotations

import math

import numpy as np

BC_INTERIOR, BC_INFLOW, BC_OUTFLOW, BC_WALL = 0, 1, 2, 3
GAMMA = 5.0 / 3.0          # monatomic gas (argon), three translational DOF
R_GAS = 0.5


# --------------------------------------------------------------------------
# splitmix64 (Steele, Lea, Flood 2014): the seeded stream behind every choice
# --------------------------------------------------------------------------
class SplitMix64:
    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def bit(self) -> int:
        return self.next_u64() >> 63


# --------------------------------------------------------------------------
# physical parameters -> model inputs
# --------------------------------------------------------------------------
def vhs_mu_ref(kn: float, omega: float, l_ref: float) -> float:
    """Reference viscosity of a VHS gas (alpha = 1) whose mean free path at
    rho = T = 1 is kn * l_ref, in units with sqrt(2 R T_inf) = 1."""
    return 15.0 * math.sqrt(math.pi) / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega)) * kn * l_ref


def sound_speed(T: float = 1.0) -> float:
    return math.sqrt(GAMMA * R_GAS * T)


# --------------------------------------------------------------------------
# 2D polygon meshes
# --------------------------------------------------------------------------
def _polygon_geometry(pts: np.ndarray):
    x, y = pts[:, 0], pts[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cross = x * yn - xn * y
    area = 0.5 * cross.sum()
    cx = ((x + xn) * cross).sum() / (6.0 * area)
    cy = ((y + yn) * cross).sum() / (6.0 * area)
    return area, np.array([cx, cy])


def build_mesh_2d(cells, classify_boundary=None):
    """Assemble face data from polygons.

    cells: list of polygons, counter-clockwise; each vertex is (vid, x, y)
    where vid identifies the vertex across periodic images and (x, y) is its
    position in that cell's own frame.
    classify_boundary(xf, n) -> (bc, bc_id) for faces with one cell.
    """
    nc = len(cells)
    vol = np.zeros(nc)
    cen = np.zeros((nc, 2))
    edges = {}
    for c, poly in enumerate(cells):
        pts = np.array([[p[1], p[2]] for p in poly], dtype=np.float64)
        a, g = _polygon_geometry(pts)
        if a <= 0:
            raise ValueError(f"cell {c} is not counter-clockwise")
        vol[c], cen[c] = a, g
        m = len(poly)
        for e in range(m):
            va, vb = poly[e], poly[(e + 1) % m]
            key = (min(va[0], vb[0]), max(va[0], vb[0]))
            edges.setdefault(key, []).append((c, np.array(va[1:]), np.array(vb[1:])))
    fc, fn, fa, fx, fs, fbc, fid = [], [], [], [], [], [], []
    for key in sorted(edges, key=lambda k: tuple(sorted(e[0] for e in edges[k])) + k):
        ent = sorted(edges[key], key=lambda e: e[0])
        c0, pa, pb = ent[0]
        d = pb - pa
        length = float(np.hypot(d[0], d[1]))
        normal = np.array([d[1], -d[0]]) / length  # outward for a CCW polygon
        mid = 0.5 * (pa + pb)
        if len(ent) == 2:
            c1, qa, qb = ent[1]
            shift = mid - 0.5 * (qa + qb)
            fc.append((c0, c1)); fbc.append(BC_INTERIOR); fid.append(0)
        elif len(ent) == 1:
            shift = np.zeros(2)
            if classify_boundary is None:
                raise ValueError("boundary edge in a mesh declared closed")
            bc, bid = classify_boundary(mid, normal)
            fc.append((c0, -1)); fbc.append(bc); fid.append(bid)
        else:
            raise ValueError("edge shared by more than two cells")
        fn.append(normal); fa.append(length); fx.append(mid); fs.append(shift)
    return dict(
        dim=2,
        cell_volume=vol,
        cell_centroid=cen,
        face_cells=np.array(fc, dtype=np.int32).reshape(-1, 2),
        face_normal=np.array(fn).reshape(-1, 2),
        face_area=np.array(fa),
        face_centroid=np.array(fx).reshape(-1, 2),
        face_shift=np.array(fs).reshape(-1, 2),
        face_bc=np.array(fbc, dtype=np.int32),
        face_bc_id=np.array(fid, dtype=np.int32),
    )


def periodic_triangles(nx=20, ny=10, lx=2.0, ly=1.0, seed=0, split="random"):
    """nx*ny quads on [0,lx]x[0,ly], each cut on a diagonal chosen by the
    seeded stream (split='random'), or all on the same one ('up'/'down').
    Periodic in both directions."""
    rng = SplitMix64(seed)
    dx, dy = lx / nx, ly / ny

    def v(i, j):
        return ((i % nx) * ny + (j % ny), i * dx, j * dy)

    cells = []
    for i in range(nx):
        for j in range(ny):
            p00, p10, p11, p01 = v(i, j), v(i + 1, j), v(i + 1, j + 1), v(i, j + 1)
            if split == "random":
                diag = rng.bit()
            else:
                diag = 0 if split == "up" else 1
            if diag == 0:   # cut p00 -- p11
                cells.append([p00, p10, p11]); cells.append([p00, p11, p01])
            else:           # cut p10 -- p01
                cells.append([p00, p10, p01]); cells.append([p10, p11, p01])
    return build_mesh_2d(cells)


def periodic_quads(nx, ny, lx=1.0, ly=1.0):
    dx, dy = lx / nx, ly / ny

    def v(i, j):
        return ((i % nx) * ny + (j % ny), i * dx, j * dy)

    cells = [[v(i, j), v(i + 1, j), v(i + 1, j + 1), v(i, j + 1)]
             for i in range(nx) for j in range(ny)]
    return build_mesh_2d(cells)


def channel_quads(nx, ny, lx=1.0, ly=1.0, y_bc=(BC_WALL, 1)):
    """Quads periodic in x, bounded in y by faces of type y_bc."""
    dx, dy = lx / nx, ly / ny

    def v(i, j):
        return ((i % nx) * (ny + 1) + j, i * dx, j * dy)

    cells = [[v(i, j), v(i + 1, j), v(i + 1, j + 1), v(i, j + 1)]
             for i in range(nx) for j in range(ny)]
    return build_mesh_2d(cells, classify_boundary=lambda xf, n: y_bc)


def cylinder_ogrid(n_theta=200, n_r=95, r_wall=1.0, r_far=15.0, h_first=1e-3,
                   n_tri_rings=5, u_inf=(1.0, 0.0), seed=0):
    """O-grid around a cylinder of radius r_wall out to r_far.  Radial spacing
    grows geometrically from h_first at the wall.  The outer n_tri_rings rings
    are cut into triangles on seeded diagonals.  Boundary faces: wall (3, id 1)
    on the cylinder; on the far field inflow (1, id 0) where u_inf . n < 0,
    else outflow (2, id 0)."""
    rng = SplitMix64(seed)
    span = r_far - r_wall
    # growth ratio g with h (g^n - 1)/(g - 1) = span
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        g = 0.5 * (lo + hi)
        s = h_first * (g ** n_r - 1.0) / (g - 1.0)
        lo, hi = (g, hi) if s < span else (lo, g)
    radii = np.empty(n_r + 1)
    radii[0] = r_wall
    h = h_first
    for j in range(n_r):
        radii[j + 1] = radii[j] + h
        h *= g
    radii[-1] = r_far
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta

    def v(i, j):
        ii = i % n_theta
        return (j * n_theta + ii, radii[j] * math.cos(th[ii]), radii[j] * math.sin(th[ii]))

    cells = []
    for j in range(n_r):
        for i in range(n_theta):
            p00, p10, p11, p01 = v(i, j), v(i, j + 1), v(i + 1, j + 1), v(i + 1, j)
            # (r, theta) ordering: r outward then theta forward is CCW
            if j >= n_r - n_tri_rings:
                if rng.bit() == 0:
                    cells.append([p00, p10, p11]); cells.append([p00, p11, p01])
                else:
                    cells.append([p00, p10, p01]); cells.append([p10, p11, p01])
            else:
                cells.append([p00, p10, p11, p01])
    uinf = np.asarray(u_inf, dtype=np.float64)
    r_mid = 0.5 * (r_wall + r_far)

    def classify(xf, n):
        if math.hypot(xf[0], xf[1]) < r_mid:
            return (BC_WALL, 1)
        return (BC_INFLOW, 0) if float(uinf @ n) < 0.0 else (BC_OUTFLOW, 0)

    return build_mesh_2d(cells, classify_boundary=classify)


# --------------------------------------------------------------------------
# velocity grids
# --------------------------------------------------------------------------
def trapezoid_1d(n: int, half_width: float, center: float = 0.0):
    x = center + np.linspace(-half_width, half_width, n)
    w = np.full(n, 2.0 * half_width / (n - 1))
    w[0] *= 0.5
    w[-1] *= 0.5
    return x, w


def tensor_vgrid(n, half_width, dim=2, center=None):
    """Cartesian velocity grid, trapezoid weights.  Point k = (a, b[, c]) is
    stored at k = (a * n + b) * n + c: the last axis is contiguous."""
    center = np.zeros(dim) if center is None else np.asarray(center, dtype=np.float64)
    axes = [trapezoid_1d(n, half_width, center[d]) for d in range(dim)]
    grids = np.meshgrid(*[a[0] for a in axes], indexing="ij")
    wg = np.meshgrid(*[a[1] for a in axes], indexing="ij")
    u = np.stack([g.reshape(-1) for g in grids], axis=1)
    w = np.prod(np.stack([g.reshape(-1) for g in wg], axis=1), axis=1)
    return dict(dim=dim, u=np.ascontiguousarray(u), w=np.ascontiguousarray(w))


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def gas_params(Pr, omega, mu_ref, cfl=0.8, limiter=1, limiter_k=1.0, bc_prim=None,
               dt_override=0.0, dim=2):
    if bc_prim is None:
        bc_prim = np.zeros((1, dim + 2)); bc_prim[0, 0] = 1.0; bc_prim[0, -1] = 1.0
    return dict(Pr=float(Pr), omega=float(omega), mu_ref=float(mu_ref), cfl=float(cfl),
                dt_override=float(dt_override), limiter=int(limiter), limiter_k=float(limiter_k),
                bc_prim=np.ascontiguousarray(np.asarray(bc_prim, dtype=np.float64)))


def case_periodic_wave(nx=20, ny=10, nv=28, half_width=6.0, kn=0.1, seed=0, Pr=1.0,
                       omega=0.5, amp=0.1, limiter=1, split="random"):
    """2D plain case: 400 triangles (20x10 quads cut on seeded diagonals) on
    [0,2]x[0,1], periodic; 28x28 trapezoid velocity grid on [-6,6]^2; BGK,
    Kn = 0.1; rho = 1 + amp sin(pi x), U = 0, T = 1; CFL 0.8."""
    mesh = periodic_triangles(nx, ny, 2.0, 1.0, seed=seed, split=split)
    vg = tensor_vgrid(nv, half_width, 2)
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 1.0), limiter=limiter)
    x = mesh["cell_centroid"][:, 0]
    prim0 = np.zeros((len(x), 4))
    prim0[:, 0] = 1.0 + amp * np.sin(math.pi * x)
    prim0[:, 3] = 1.0
    return dict(name=f"periodic_tri_{2*nx*ny}_v{nv}x{nv}", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)


def case_cylinder(n_theta=200, n_r=95, n_tri_rings=5, nv=60, half_width=15.0, ma=5.0, kn=0.1,
                  Pr=2.0 / 3.0, omega=0.81, t_wall=1.0, h_first=1e-3, r_far=15.0, seed=0,
                  start="potential", wall_layer=0.2):
    """2D hypersonic cylinder: unit-radius cylinder, far field radius 15,
    200 x 95 O-grid with the outer 5 rings cut into triangles (20,000 cells),
    first layer 1e-3; Shakhov Pr = 2/3, Ma = 5, Kn = 0.1 on the diameter,
    isothermal wall at T_inf; 60 x 60 trapezoid grid on [-15,15]^2.

    start='potential': rho = T = 1 with the incompressible potential flow
    around the cylinder, brought to rest at the wall over a layer of
    thickness wall_layer (U * (1 - exp(-(r - 1)/wall_layer))).
    start='freestream': uniform free stream (impulsive start; the leeward
    first-layer cells empty within tens of steps)."""
    u_inf = ma * sound_speed(1.0)
    mesh = cylinder_ogrid(n_theta, n_r, 1.0, r_far, h_first, n_tri_rings, (u_inf, 0.0), seed)
    vg = tensor_vgrid(nv, half_width, 2)
    bc = np.array([[1.0, u_inf, 0.0, 1.0],       # free stream
                   [1.0, 0.0, 0.0, t_wall]])     # wall (rho unused)
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 2.0), bc_prim=bc)
    nc = len(mesh["cell_volume"])
    prim0 = np.tile(bc[0], (nc, 1))
    if start == "potential":
        x = mesh["cell_centroid"]
        r = np.hypot(x[:, 0], x[:, 1])
        th = np.arctan2(x[:, 1], x[:, 0])
        ur = u_inf * (1.0 - 1.0 / r ** 2) * np.cos(th)
        ut = -u_inf * (1.0 + 1.0 / r ** 2) * np.sin(th)
        damp = 1.0 - np.exp(-(r - 1.0) / wall_layer)
        prim0[:, 1] = (ur * np.cos(th) - ut * np.sin(th)) * damp
        prim0[:, 2] = (ur * np.sin(th) + ut * np.cos(th)) * damp
    elif start != "freestream":
        raise ValueError(start)
    return dict(name=f"cylinder_{nc}_v{nv}x{nv}", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)


def case_cylinder_small(n_theta=40, n_r=16, n_tri_rings=2, nv=24, half_width=15.0, ma=5.0, kn=0.1,
                        h_first=1e-2, seed=0, Pr=2.0 / 3.0, start="potential"):
    """Cut-down of the hypersonic cylinder (same physics, wall, far field and
    mixed quad/triangle mesh) that the oracle steps in about a second."""
    return case_cylinder(n_theta=n_theta, n_r=n_r, n_tri_rings=n_tri_rings, nv=nv, half_width=half_width, ma=ma,
                         kn=kn, h_first=h_first, seed=seed, Pr=Pr, start=start)


def n_comp(dim: int) -> int:
    """Stored reduced distributions per (cell, velocity): h and b in 2D
    (one internal velocity component), h only in 3D (no internal component
    for a monatomic gas, so b is identically zero)."""
    return 2 if dim == 2 else 1


# --------------------------------------------------------------------------
# 3D polyhedral meshes
# --------------------------------------------------------------------------
def _poly_area_centroid(P):
    """Area vector (right-hand rule over the vertex order) and centroid of a
    planar polygon in 3D, by a fan of triangles."""
    a = np.zeros(3)
    c = np.zeros(3)
    for t in range(1, len(P) - 1):
        at = 0.5 * np.cross(P[t] - P[0], P[t + 1] - P[0])
        w = np.linalg.norm(at)
        a += at
        c += w * (P[0] + P[t] + P[t + 1]) / 3.0
    return a, c / max(np.linalg.norm(a), 1e-300)


def build_mesh_3d(cells, classify_boundary=None):
    """Assemble face data from polyhedra.

    cells: list of polyhedra; each is a list of faces, each face a list of
    vertices (vid, x, y, z) ordered counter-clockwise seen from outside the
    cell; vid identifies the vertex across periodic images and (x, y, z) is
    its position in that cell's own frame.
    """
    nc = len(cells)
    vol = np.zeros(nc)
    cen = np.zeros((nc, 3))
    faces = {}
    for c, poly in enumerate(cells):
        pts = np.array([[v[1], v[2], v[3]] for f in poly for v in f])
        ref = pts.mean(axis=0)
        V = 0.0
        C = np.zeros(3)
        for f in poly:
            P = np.array([[v[1], v[2], v[3]] for v in f])
            for t in range(1, len(P) - 1):
                tv = np.dot(P[0] - ref, np.cross(P[t] - ref, P[t + 1] - ref)) / 6.0
                V += tv
                C += tv * (ref + P[0] + P[t] + P[t + 1]) / 4.0
            key = tuple(sorted(v[0] for v in f))
            faces.setdefault(key, []).append((c, P))
        if V <= 0:
            raise ValueError(f"cell {c} has non-positive volume (faces not outward)")
        vol[c], cen[c] = V, C / V
    fc, fn, fa, fx, fs, fbc, fid = [], [], [], [], [], [], []
    for key in sorted(faces, key=lambda k: tuple(sorted(e[0] for e in faces[k])) + k):
        ent = sorted(faces[key], key=lambda e: e[0])
        c0, P0 = ent[0]
        av, xc = _poly_area_centroid(P0)
        area = float(np.linalg.norm(av))
        normal = av / area
        if len(ent) == 2:
            c1, P1 = ent[1]
            _, x1 = _poly_area_centroid(P1)
            shift = xc - x1
            fc.append((c0, c1)); fbc.append(BC_INTERIOR); fid.append(0)
        elif len(ent) == 1:
            shift = np.zeros(3)
            if classify_boundary is None:
                raise ValueError("boundary face in a mesh declared closed")
            bc, bid = classify_boundary(xc, normal)
            fc.append((c0, -1)); fbc.append(bc); fid.append(bid)
        else:
            raise ValueError("face shared by more than two cells")
        fn.append(normal); fa.append(area); fx.append(xc); fs.append(shift)
    return dict(dim=3, cell_volume=vol, cell_centroid=cen,
                face_cells=np.array(fc, dtype=np.int32).reshape(-1, 2),
                face_normal=np.array(fn).reshape(-1, 3), face_area=np.array(fa),
                face_centroid=np.array(fx).reshape(-1, 3), face_shift=np.array(fs).reshape(-1, 3),
                face_bc=np.array(fbc, dtype=np.int32), face_bc_id=np.array(fid, dtype=np.int32))


_HEX_FACES = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (2, 3, 7, 6), (0, 4, 7, 3), (1, 2, 6, 5)]
_CUBE = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def _tet_faces(v):
    """Four outward-ordered triangles of the tetrahedron v[0..3]."""
    P = [np.array(x[1:]) for x in v]
    faces = []
    for skip in range(4):
        tri = [v[j] for j in range(4) if j != skip]
        a, b, c = (np.array(t[1:]) for t in tri)
        if np.dot(np.cross(b - a, c - a), a - P[skip]) < 0:
            tri = [tri[0], tri[2], tri[1]]
        faces.append(tri)
    return faces


def box_mesh_3d(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, kind="hex", periodic=(True, True, True),
                classify_boundary=None):
    """Box of nx*ny*nz cubes: hexahedra, 6 tetrahedra per cube (Kuhn split
    along the main diagonal, conforming between cubes), or 2 triangular
    prisms per cube.  Periodic along the flagged axes."""
    n = (nx, ny, nz)
    h = (lx / nx, ly / ny, lz / nz)

    def v(i, j, k):
        idx = [i, j, k]
        vid = 0
        for d in range(3):
            m = n[d] if periodic[d] else n[d] + 1
            vid = vid * m + (idx[d] % n[d] if periodic[d] else idx[d])
        return (vid, i * h[0], j * h[1], k * h[2])

    cells = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                cv = [v(i + a, j + b, k + c) for (a, b, c) in _CUBE]
                if kind == "hex":
                    cells.append([[cv[q] for q in f] for f in _HEX_FACES])
                elif kind == "tet":
                    import itertools
                    for perm in itertools.permutations(range(3)):
                        p = [0, 0, 0]
                        path = [tuple(p)]
                        for ax in perm:
                            p[ax] += 1
                            path.append(tuple(p))
                        tv = [v(i + a, j + b, k + c) for (a, b, c) in path]
                        cells.append(_tet_faces(tv))
                elif kind == "prism":
                    for tri in ((0, 1, 2), (0, 2, 3)):
                        bot = [cv[t] for t in tri]
                        top = [cv[t + 4] for t in tri]
                        cells.append([[bot[0], bot[2], bot[1]], [top[0], top[1], top[2]],
                                      [bot[0], bot[1], top[1], top[0]], [bot[1], bot[2], top[2], top[1]],
                                      [bot[2], bot[0], top[0], top[2]]])
                else:
                    raise ValueError(kind)
    return build_mesh_3d(cells, classify_boundary)


def case_box_wave_3d(n=3, kind="tet", nv=8, half_width=5.0, kn=0.1, Pr=2.0 / 3.0, omega=0.81, amp=0.1,
                     limiter=1):
    """3D periodic box [0,1]^3 of n^3 cubes (hex, tet or prism cells) with a
    density/temperature wave and a drift; Cartesian nv^3 velocity grid."""
    mesh = box_mesh_3d(n, n, n, kind=kind)
    vg = tensor_vgrid(nv, half_width, 3)
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 1.0), limiter=limiter, dim=3)
    x = mesh["cell_centroid"]
    prim0 = np.zeros((len(x), 5))
    prim0[:, 0] = 1.0 + amp * np.sin(2 * math.pi * x[:, 0]) * np.cos(2 * math.pi * x[:, 2])
    prim0[:, 1] = 0.1
    prim0[:, 2] = -0.05 * np.sin(2 * math.pi * x[:, 1])
    prim0[:, 3] = 0.05
    prim0[:, 4] = 1.0 + 0.5 * amp * np.cos(2 * math.pi * x[:, 1])
    return dict(name=f"box3d_{kind}_{len(x)}_v{nv}^3", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)


def case_channel_3d(n=3, kind="hex", nv=8, half_width=5.0, kn=0.1, Pr=2.0 / 3.0, omega=0.81, t_wall=1.2,
                    u_wall=0.3):
    """3D box periodic in x and y between two isothermal walls at z = 0 and
    z = 1; the top wall slides in x (moving-wall Couette start)."""
    def classify(xf, nrm):
        return (BC_WALL, 1) if xf[2] > 0.5 else (BC_WALL, 2)
    mesh = box_mesh_3d(n, n, n, kind=kind, periodic=(True, True, False), classify_boundary=classify)
    vg = tensor_vgrid(nv, half_width, 3)
    bc = np.array([[1.0, 0.0, 0.0, 0.0, 1.0],
                   [1.0, u_wall, 0.0, 0.0, t_wall],
                   [1.0, 0.0, 0.0, 0.0, 1.0]])
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 1.0), bc_prim=bc, dim=3)
    x = mesh["cell_centroid"]
    prim0 = np.zeros((len(x), 5))
    prim0[:, 0] = 1.0 + 0.05 * np.sin(2 * math.pi * x[:, 0])
    prim0[:, 4] = 1.0
    return dict(name=f"channel3d_{kind}_{len(x)}_v{nv}^3", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)


# --------------------------------------------------------------------------
# large 3D meshes from connectivity arrays (vectorised)
# --------------------------------------------------------------------------
def mesh_from_tets(X, T, classify_boundary):
    """Face data of a tetrahedral mesh given vertex coordinates X [nv][3] and
    tetrahedra T [nc][4] (any orientation).  classify_boundary(xc, n) takes
    arrays of boundary face centroids and outward normals and returns arrays
    (bc, bc_id)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64).copy()
    P = X[T]
    vol6 = np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))
    neg = vol6 < 0
    T[neg, 1], T[neg, 2] = T[neg, 2].copy(), T[neg, 1].copy()
    P = X[T]
    vol = np.abs(vol6) / 6.0
    if (vol <= 0).any():
        raise ValueError("degenerate tetrahedron")
    cen = P.mean(axis=1)
    nc = len(T)
    # the four faces of a positively oriented tetrahedron, outward
    loc = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
    F = T[:, loc].reshape(-1, 3)
    owner = np.repeat(np.arange(nc), 4)
    key = np.sort(F, axis=1)
    order = np.lexsort((owner, key[:, 2], key[:, 1], key[:, 0]))
    key, F, owner = key[order], F[order], owner[order]
    first = np.ones(len(key), dtype=bool)
    first[1:] = (key[1:] != key[:-1]).any(axis=1)
    start = np.nonzero(first)[0]
    count = np.diff(np.append(start, len(key)))
    if (count > 2).any():
        raise ValueError("face shared by more than two cells")
    Ff = F[start]
    l = owner[start]
    r = np.where(count == 2, owner[np.minimum(start + 1, len(owner) - 1)], -1)
    A = X[Ff]
    av = 0.5 * np.cross(A[:, 1] - A[:, 0], A[:, 2] - A[:, 0])
    area = np.linalg.norm(av, axis=1)
    normal = av / area[:, None]
    xc = A.mean(axis=1)
    bc = np.zeros(len(Ff), dtype=np.int32)
    bid = np.zeros(len(Ff), dtype=np.int32)
    b = r < 0
    if b.any():
        cb, ib = classify_boundary(xc[b], normal[b])
        bc[b], bid[b] = cb, ib
    return dict(dim=3, cell_volume=vol, cell_centroid=cen,
                face_cells=np.stack([l, r], 1).astype(np.int32), face_normal=normal, face_area=area,
                face_centroid=xc, face_shift=np.zeros_like(xc), face_bc=bc, face_bc_id=bid)


def prisms_to_tets(Pz):
    """Split prisms [n][6] (bottom triangle 0,1,2; top 3,4,5 above them)
    into three tetrahedra each, conformingly: every quadrilateral side is cut
    along the diagonal through its lowest global vertex index (the rule of
    Dompierre et al., which always admits a three-tetrahedron split)."""
    Pz = np.asarray(Pz, dtype=np.int64)
    p = np.argmin(Pz, axis=1)
    q = p % 3
    rot = np.stack([q, (q + 1) % 3, (q + 2) % 3], 1)
    top = (p >= 3)[:, None]
    perm = np.where(top, np.concatenate([rot + 3, rot], 1), np.concatenate([rot, rot + 3], 1))
    I = np.take_along_axis(Pz, perm, axis=1)
    a = np.minimum(I[:, 1], I[:, 5]) < np.minimum(I[:, 2], I[:, 4])
    tA = np.stack([I[:, [0, 1, 2, 5]], I[:, [0, 1, 5, 4]], I[:, [0, 4, 5, 3]]], 1)
    tB = np.stack([I[:, [0, 1, 2, 4]], I[:, [0, 4, 2, 5]], I[:, [0, 4, 5, 3]]], 1)
    return np.where(a[:, None, None], tA, tB).reshape(-1, 4)


def cubed_sphere_shell(n, n_r, r_wall=1.0, r_far=6.0, h_first=5e-3):
    """Vertices and prisms of a spherical shell: the six faces of a cube,
    each an n x n grid of equal-angle points projected onto the sphere and
    cut into triangles, extruded over n_r layers whose thickness grows
    geometrically from h_first at the wall to r_far."""
    span = r_far - r_wall
    lo, hi = 1.0 + 1e-12, 3.0
    for _ in range(200):
        g = 0.5 * (lo + hi)
        s = h_first * (g ** n_r - 1.0) / (g - 1.0)
        lo, hi = (g, hi) if s < span else (lo, g)
    radii = r_wall + h_first * (g ** np.arange(n_r + 1) - 1.0) / (g - 1.0)
    radii[-1] = r_far
    t = np.tan(-0.25 * math.pi + 0.5 * math.pi * np.arange(n + 1) / n)
    pts, tris = [], []
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            a, b = np.meshgrid(t, t, indexing="ij")
            v = np.zeros((n + 1, n + 1, 3))
            v[..., ax] = sgn
            v[..., (ax + 1) % 3] = a
            v[..., (ax + 2) % 3] = b
            v /= np.linalg.norm(v, axis=2, keepdims=True)
            base = len(pts) * 0 + sum(len(x) for x in pts)
            pts.append(v.reshape(-1, 3))
            idx = base + np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
            q00, q10, q11, q01 = idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:], idx[:-1, 1:]
            tris.append(np.stack([q00, q10, q11], -1).reshape(-1, 3))
            tris.append(np.stack([q00, q11, q01], -1).reshape(-1, 3))
    S = np.concatenate(pts)
    # merge the points shared by neighbouring cube faces
    _, uniq, inv = np.unique(np.round(S, 12), axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    S = S[uniq]
    tri = inv[np.concatenate(tris)]
    ns = len(S)
    X = (radii[:, None, None] * S[None, :, :]).reshape(-1, 3)
    layers = np.arange(n_r)[:, None, None] * ns
    prisms = np.concatenate([tri[None] + layers, tri[None] + layers + ns], axis=2).reshape(-1, 6)
    return X, prisms


def case_sphere(n=8, n_r=22, nv=24, half_width=10.0, ma=4.0, kn=0.05, Pr=0.72, omega=0.81, t_wall=1.0,
                r_far=6.0, h_first=5e-3, wall_layer=0.2, kind="tet"):
    """3D sphere: a cubed-sphere shell around the unit sphere out to radius
    6, n x n points per cube face, n_r layers from a 5e-3 first layer, each
    prism cut into three tetrahedra (36 n^2 n_r cells: 50,688 by default);
    Shakhov Pr = 0.72, Ma = 4, Kn = 0.05 on the diameter, isothermal wall at
    T_inf; 24^3 trapezoid grid on [-10,10]^3.  Start: rho = T = 1 with the
    potential flow around the sphere brought to rest over a wall layer.
    kind='hex': the same shell as hexahedra (6 n^2 n_r cells; n=16, n_r=33
    also gives 50,688), the paper's own cell type for its sphere."""
    u_inf = ma * sound_speed(1.0)
    r_mid = 0.5 * (1.0 + r_far)
    if kind == "hex":
        # straight lines from the sphere to the far field, first layer
        # h_first (the shell builder takes it relative to the line length)
        X, hexes, _ = lifting_body_shell(n, n_r, 0, axes=(1.0, 1.0, 1.0), z_lower=1.0, r_far=r_far,
                                         h_first=h_first / (r_far - 1.0))
    else:
        X, prisms = cubed_sphere_shell(n, n_r, 1.0, r_far, h_first)
        T = prisms_to_tets(prisms)
    uvec = np.array([u_inf, 0.0, 0.0])

    def classify(xc, nrm):
        wall = np.linalg.norm(xc, axis=1) < r_mid
        bc = np.where(wall, BC_WALL, np.where(nrm @ uvec < 0.0, BC_INFLOW, BC_OUTFLOW)).astype(np.int32)
        return bc, np.where(wall, 1, 0).astype(np.int32)

    mesh = mesh_from_cells(X, classify, hexes=hexes) if kind == "hex" else mesh_from_tets(X, T, classify)
    vg = tensor_vgrid(nv, half_width, 3)
    bc = np.array([[1.0, u_inf, 0.0, 0.0, 1.0],
                   [1.0, 0.0, 0.0, 0.0, t_wall]])
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 2.0), bc_prim=bc, dim=3)
    x = mesh["cell_centroid"]
    r = np.linalg.norm(x, axis=1)
    # potential flow past the unit sphere, phi = U x (1 + 1/(2 r^3)), brought
    # to rest at the wall over wall_layer
    vel = u_inf * (1.0 + 0.5 / r ** 3)[:, None] * np.array([1.0, 0.0, 0.0]) \
        - (1.5 * u_inf * x[:, 0] / r ** 5)[:, None] * x
    damp = 1.0 - np.exp(-(r - 1.0) / wall_layer)
    prim0 = np.tile(bc[0], (len(x), 1))
    prim0[:, 1:4] = vel * damp[:, None]
    return dict(name=f"sphere_{len(x)}{kind}_v{nv}^3", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)


def mesh_from_cells(X, classify_boundary, tets=None, prisms=None, hexes=None):
    """Face data of a mesh of tetrahedra [n][4], prisms [n][6] (bottom
    triangle 0,1,2, top 3,4,5 above) and hexahedra [n][8] (bottom quad 0..3,
    top 4..7 above), vectorised.  Face area vectors are exact for bilinear
    quadrilaterals (half the cross product of the diagonals) and oriented out
    of the first cell; cell volumes and centroids come from tetrahedra
    between the vertex average and the face triangles."""
    X = np.asarray(X, dtype=np.float64)
    groups = []
    if tets is not None:
        groups.append((np.asarray(tets, np.int64), [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]))
    if prisms is not None:
        groups.append((np.asarray(prisms, np.int64), [(0, 2, 1), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)]))
    if hexes is not None:
        groups.append((np.asarray(hexes, np.int64), [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5),
                                                     (2, 3, 7, 6), (3, 0, 4, 7)]))
    tri_f, tri_o, quad_f, quad_o = [], [], [], []
    vols, cens = [], []
    off = 0
    for C, loc in groups:
        G = X[C].mean(axis=1)
        V = np.zeros(len(C))
        M = np.zeros((len(C), 3))
        for fl in loc:
            F = C[:, list(fl)]
            P = X[F]
            # orient outward (cells are convex): normal away from the vertex average
            if len(fl) == 3:
                av = 0.5 * np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
            else:
                av = 0.5 * np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 1])
            flip = np.einsum("ij,ij->i", av, P.mean(axis=1) - G) < 0
            F = np.where(flip[:, None], F[:, ::-1], F)
            P = X[F]
            tris = [(0, 1, 2)] if len(fl) == 3 else [(0, 1, 2), (0, 2, 3)]
            for a, b, c in tris:
                tv = np.einsum("ij,ij->i", P[:, a] - G, np.cross(P[:, b] - G, P[:, c] - G)) / 6.0
                V += tv
                M += tv[:, None] * (G + P[:, a] + P[:, b] + P[:, c]) / 4.0
            owner = off + np.arange(len(C))
            (tri_f if len(fl) == 3 else quad_f).append(F)
            (tri_o if len(fl) == 3 else quad_o).append(owner)
        if (V <= 0).any():
            raise ValueError("cell with non-positive volume")
        vols.append(V)
        cens.append(M / V[:, None])
        off += len(C)
    vol = np.concatenate(vols)
    cen = np.concatenate(cens)
    out = {k: [] for k in ("l", "r", "av", "xc")}
    for Fs, Os in ((tri_f, tri_o), (quad_f, quad_o)):
        if not Fs:
            continue
        F = np.concatenate(Fs)
        own = np.concatenate(Os)
        key = np.sort(F, axis=1)
        order = np.lexsort((own,) + tuple(key[:, j] for j in range(key.shape[1] - 1, -1, -1)))
        key, F, own = key[order], F[order], own[order]
        first = np.ones(len(key), dtype=bool)
        first[1:] = (key[1:] != key[:-1]).any(axis=1)
        start = np.nonzero(first)[0]
        count = np.diff(np.append(start, len(key)))
        if (count > 2).any():
            raise ValueError("face shared by more than two cells")
        Ff = F[start]
        P = X[Ff]
        if F.shape[1] == 3:
            av = 0.5 * np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
            xc = P.mean(axis=1)
        else:
            av = 0.5 * np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 1])
            a1 = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
            a2 = 0.5 * np.linalg.norm(np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]), axis=1)
            c1 = (P[:, 0] + P[:, 1] + P[:, 2]) / 3.0
            c2 = (P[:, 0] + P[:, 2] + P[:, 3]) / 3.0
            xc = (a1[:, None] * c1 + a2[:, None] * c2) / (a1 + a2)[:, None]
        out["l"].append(own[start])
        out["r"].append(np.where(count == 2, own[np.minimum(start + 1, len(own) - 1)], -1))
        out["av"].append(av)
        out["xc"].append(xc)
    l, r = np.concatenate(out["l"]), np.concatenate(out["r"])
    av, xc = np.concatenate(out["av"]), np.concatenate(out["xc"])
    area = np.linalg.norm(av, axis=1)
    normal = av / area[:, None]
    bc = np.zeros(len(l), dtype=np.int32)
    bid = np.zeros(len(l), dtype=np.int32)
    b = r < 0
    if b.any():
        cb, ib = classify_boundary(xc[b], normal[b])
        bc[b], bid[b] = cb, ib
    return dict(dim=3, cell_volume=vol, cell_centroid=cen, face_cells=np.stack([l, r], 1).astype(np.int32),
                face_normal=normal, face_area=area, face_centroid=xc, face_shift=np.zeros_like(xc),
                face_bc=bc, face_bc_id=bid)


def lifting_body_shell(n, n_r, n_prism_columns=0, axes=(3.0, 1.2, 0.6), z_lower=0.35, r_far=12.0, h_first=5e-3):
    """Hexahedra and prisms around a synthetic lifting body: an ellipsoid with
    semi-axes `axes` above z = 0 and a flatter lower surface (z semi-axis
    z_lower).  The six faces of a cube, n x n equal-angle points each, are
    projected onto the body and joined by straight lines to a far-field
    sphere of radius r_far, n_r layers growing geometrically from h_first
    (relative to the local line length): 6 n^2 n_r hexahedra.  The
    n_prism_columns radial columns nearest the two poles (the z axis) are
    each cut into two prisms along a diagonal of their quadrilaterals (whole
    columns, so that the cut faces match between layers): 6 n^2 n_r +
    n_prism_columns n_r cells."""
    lo, hi = 1.0 + 1e-12, 3.0
    for _ in range(200):
        g = 0.5 * (lo + hi)
        s = h_first * (g ** n_r - 1.0) / (g - 1.0)
        lo, hi = (g, hi) if s < 1.0 else (lo, g)
    eta = h_first * (g ** np.arange(n_r + 1) - 1.0) / (g - 1.0)
    eta[-1] = 1.0
    t = np.tan(-0.25 * math.pi + 0.5 * math.pi * np.arange(n + 1) / n)
    pts, quads = [], []
    base = 0
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            a, b = np.meshgrid(t, t, indexing="ij")
            v = np.zeros((n + 1, n + 1, 3))
            v[..., ax] = sgn
            v[..., (ax + 1) % 3] = a
            v[..., (ax + 2) % 3] = b
            v /= np.linalg.norm(v, axis=2, keepdims=True)
            pts.append(v.reshape(-1, 3))
            idx = base + np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
            quads.append(np.stack([idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:], idx[:-1, 1:]], -1).reshape(-1, 4))
            base += (n + 1) * (n + 1)
    S = np.concatenate(pts)
    _, uniq, inv = np.unique(np.round(S, 12), axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    S = S[uniq]
    Q = inv[np.concatenate(quads)]
    ns = len(S)
    scale = np.tile(np.asarray(axes, dtype=np.float64), (ns, 1))
    scale[S[:, 2] < 0, 2] = z_lower
    body = S * scale
    far = S * r_far
    X = (body[None] + eta[:, None, None] * (far - body)[None]).reshape(-1, 3)
    # columns nearest the poles become prisms (ties broken by column index)
    pole = 1.0 - np.abs(S[Q].mean(axis=1)[:, 2])
    order = np.lexsort((np.arange(len(Q)), pole))
    split = np.zeros(len(Q), dtype=bool)
    split[order[:n_prism_columns]] = True
    layers = np.arange(n_r)[:, None, None] * ns
    Qh, Qp = Q[~split], Q[split]
    hexes = np.concatenate([Qh[None] + layers, Qh[None] + layers + ns], axis=2).reshape(-1, 8)
    prisms = None
    if len(Qp):
        tri = np.concatenate([Qp[:, [0, 1, 2]], Qp[:, [0, 2, 3]]])
        prisms = np.concatenate([tri[None] + layers, tri[None] + layers + ns], axis=2).reshape(-1, 6)
    return X, hexes, prisms


def octree_vgrid(n_base, half_width, levels, n_keep=None):
    """Unstructured velocity set: an n_base^3 Cartesian partition of
    [-half_width, half_width]^3 refined level by level: at each level
    (centres, radius) the cells whose centre lies within radius of one of
    the centres (e.g. the free-stream and wall Maxwellians) are split into
    eight.  The points are the cell centres and the weights the cell volumes
    (Section 2.3, unstructured velocity meshes).  n_keep trims the set to
    that many points by dropping the ones farthest from the origin."""
    h = 2.0 * half_width / n_base
    g = -half_width + h * (np.arange(n_base) + 0.5)
    C = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    H = np.full(len(C), h)
    sub = np.array([[a, b, c] for a in (-0.25, 0.25) for b in (-0.25, 0.25) for c in (-0.25, 0.25)])
    for centres, radius in levels:
        near = np.zeros(len(C), dtype=bool)
        for c in centres:
            near |= np.linalg.norm(C - np.asarray(c)[None], axis=1) < radius
        fine = (C[near][:, None, :] + sub[None] * H[near][:, None, None]).reshape(-1, 3)
        C = np.concatenate([C[~near], fine])
        H = np.concatenate([H[~near], np.repeat(0.5 * H[near], 8)])
    w = H ** 3
    if n_keep is not None and n_keep < len(w):
        keep = np.sort(np.lexsort((np.arange(len(w)), np.linalg.norm(C, axis=1)))[:n_keep])
        C, w = C[keep], w[keep]
    return dict(dim=3, u=np.ascontiguousarray(C), w=np.ascontiguousarray(w))


def case_lifting_body(n=32, n_r=163, n_prism_columns=351, ma=8.0, kn=0.01, Pr=0.72, omega=0.81, t_wall=5.39,
                      aoa_deg=20.0, n_base=14, half_width=15.0, refine=(6.5, 2.2), n_vel=4548, closed=False,
                      start="layer", wall_layer=0.5):
    """X38-sized synthetic blunt body: 1,058,685 cells (hexahedra, and the
    351 radial columns nearest the poles as prisms) around a lifting body
    out to a radius-12 far field; Ma 8 at 20 degrees angle of attack,
    Kn 0.01, Shakhov Pr 0.72, wall at 5.39 T_inf; an unstructured velocity
    set of 4,548 points: 14^3 cells of [-15,15]^3, those within 6.5 of the
    free-stream or the wall velocity split once, those within 2.2 of the
    free-stream velocity split again.
    closed=True turns the far field into a resting wall at T_inf (a closed
    vessel, whose mass the scheme conserves exactly at any size).  Start:
    'layer' (default) the free stream brought to rest towards the body, as
    U_inf (1 - exp(-(F - 1)/wall_layer)) with F the body's ellipsoid
    function (1 on the surface); 'freestream' the uniform free stream
    (impulsive: the first layer empties within tens of steps); 'rest' gas
    at rest at T_inf."""
    u_inf = ma * sound_speed(1.0)
    a = math.radians(aoa_deg)
    U = np.array([u_inf * math.cos(a), 0.0, u_inf * math.sin(a)])
    X, hexes, prisms = lifting_body_shell(n, n_r, n_prism_columns)

    def classify(xc, nrm):
        body = np.linalg.norm(xc, axis=1) < 6.0
        if closed:
            return np.full(len(xc), BC_WALL, np.int32), np.where(body, 1, 2).astype(np.int32)
        far = np.where(nrm @ U < 0.0, BC_INFLOW, BC_OUTFLOW)
        return np.where(body, BC_WALL, far).astype(np.int32), np.where(body, 1, 0).astype(np.int32)

    mesh = mesh_from_cells(X, classify, prisms=prisms, hexes=hexes)
    vg = octree_vgrid(n_base, half_width, [([U, np.zeros(3)], refine[0]), ([U], refine[1])], n_vel)
    bc = np.array([[1.0, U[0], U[1], U[2], 1.0],
                   [1.0, 0.0, 0.0, 0.0, t_wall],
                   [1.0, 0.0, 0.0, 0.0, 1.0]])
    gas = gas_params(Pr, omega, vhs_mu_ref(kn, omega, 6.0), bc_prim=bc, dim=3)
    if start not in ("layer", "freestream", "rest"):
        raise ValueError(start)
    prim0 = np.tile(bc[2] if start == "rest" else bc[0], (len(mesh["cell_volume"]), 1))
    if start == "layer":
        x = mesh["cell_centroid"]
        cz = np.where(x[:, 2] < 0.0, 0.35, 0.6)
        F = np.sqrt((x[:, 0] / 3.0) ** 2 + (x[:, 1] / 1.2) ** 2 + (x[:, 2] / cz) ** 2)
        prim0[:, 1:4] *= (1.0 - np.exp(-np.maximum(F - 1.0, 0.0) / wall_layer))[:, None]
    nc, nv = len(mesh["cell_volume"]), len(vg["w"])
    return dict(name=f"liftingbody_{nc}_v{nv}", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)
