"""FP64 CPU oracle of the memory-saving UGKS step (ctypes loader).

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package.  It shares no code with the HIP
library in paper_2412_06546_amd/; the two meet only in the seeded inputs of
paper_2412_06546_amd.cases.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ugks_oracle.c")
_LIB = os.path.join(_HERE, "libugks_oracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Input(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_cells", C.c_int), ("n_faces", C.c_int), ("n_vel", C.c_int),
        ("cell_volume", _dp), ("cell_centroid", _dp),
        ("face_cells", _ip),
        ("face_normal", _dp), ("face_area", _dp), ("face_centroid", _dp), ("face_shift", _dp),
        ("face_bc", _ip), ("face_bc_id", _ip),
        ("u", _dp), ("w", _dp),
        ("Pr", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double), ("cfl", C.c_double),
        ("dt_override", C.c_double), ("limiter_k", C.c_double),
        ("limiter", C.c_int), ("n_bc", C.c_int),
        ("bc_prim", _dp), ("prim0", _dp),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (the paper's optimisation level) and
    OpenMP over cells."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Input)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_nstep.restype = C.c_long
        L.orc_nstep.argtypes = [C.c_void_p]
        L.orc_get.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_set_f.argtypes = [C.c_void_p, _dp]
        L.orc_residual.argtypes = [C.c_void_p, _dp]
        L.orc_set_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_n_wall.restype = C.c_int
        L.orc_n_wall.argtypes = [C.c_void_p]
        L.orc_wall_flux.argtypes = [C.c_void_p, _dp]
        L.orc_time_integrals.argtypes = [C.c_double, C.c_double, _dp]
        L.orc_prim_of_cons.argtypes = [C.c_int, _dp, _dp]
        L.orc_cons_of_prim.argtypes = [C.c_int, _dp, _dp]
        L.orc_reduced_eq.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_half_merge.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_slope_of_g0.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_time_slope_of_g0.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_venkat.restype = C.c_double
        L.orc_venkat.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_gauss_hermite.restype = C.c_int
        L.orc_gauss_hermite.argtypes = [_dp, _dp]
        L.orc_macro_gradients.argtypes = [C.c_void_p, _dp, _ip]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class Oracle:
    """One flow case advanced by the CPU oracle."""

    def __init__(self, case, omp_threads: int | None = None):
        L = lib()
        self.threads = L.orc_set_threads(int(omp_threads) if omp_threads else 0)
        m, vg, gas = case["mesh"], case["vgrid"], case["gas"]
        self.dim = int(m["dim"])
        self.nc = len(m["cell_volume"])
        self.nv = len(vg["w"])
        self.ncomp = 2 if self.dim == 2 else 1
        keep = []

        def d(x):
            a, p = _d(x); keep.append(a); return p

        def i(x):
            a, p = _i(x); keep.append(a); return p

        inp = _Input()
        inp.dim, inp.n_cells, inp.n_faces, inp.n_vel = self.dim, self.nc, len(m["face_area"]), self.nv
        inp.cell_volume, inp.cell_centroid = d(m["cell_volume"]), d(m["cell_centroid"])
        inp.face_cells = i(m["face_cells"])
        inp.face_normal, inp.face_area = d(m["face_normal"]), d(m["face_area"])
        inp.face_centroid, inp.face_shift = d(m["face_centroid"]), d(m["face_shift"])
        inp.face_bc, inp.face_bc_id = i(m["face_bc"]), i(m["face_bc_id"])
        inp.u, inp.w = d(vg["u"]), d(vg["w"])
        for k in ("Pr", "omega", "mu_ref", "cfl", "dt_override", "limiter_k"):
            setattr(inp, k, float(gas[k]))
        inp.limiter = int(gas["limiter"])
        bc = np.asarray(gas["bc_prim"], dtype=np.float64)
        inp.n_bc = bc.shape[0]
        inp.bc_prim = d(bc)
        inp.prim0 = d(case["prim0"])
        self._h = L.orc_create(C.byref(inp))
        if not self._h:
            raise RuntimeError("oracle rejected the case")
        self._L = L

    def __del__(self):
        if getattr(self, "_h", None):
            self._L.orc_destroy(self._h)
            self._h = None

    @property
    def dt(self) -> float:
        return self._L.orc_dt(self._h)

    def set_threads(self, n: int) -> int:
        """OpenMP threads of the oracle's loops from now on."""
        self.threads = self._L.orc_set_threads(int(n))
        return self.threads

    @property
    def nstep(self) -> int:
        return self._L.orc_nstep(self._h)

    def step(self, n: int = 1):
        self._L.orc_step(self._h, int(n))

    def macros(self):
        W = np.zeros((self.nc, self.dim + 2))
        q = np.zeros((self.nc, self.dim))
        self._L.orc_get(self._h, W.ctypes.data_as(_dp), q.ctypes.data_as(_dp), None)
        return W, q

    def f(self):
        f = np.zeros((self.nc, self.ncomp, self.nv))
        self._L.orc_get(self._h, None, None, f.ctypes.data_as(_dp))
        return f

    def set_f(self, f):
        a, p = _d(f)
        assert a.shape == (self.nc, self.ncomp, self.nv)
        self._L.orc_set_f(self._h, p)

    def macro_gradients(self):
        """Limited gradients of W for the current state (the macroscopic reconstruction of Algorithm 1),
        [nc][dim + 2][dim], and per cell whether it fell back to first
        order (a reconstructed face state not physical)."""
        g = np.zeros((self.nc, self.dim + 2, self.dim))
        bad = np.zeros(self.nc, dtype=np.int32)
        self._L.orc_macro_gradients(self._h, g.ctypes.data_as(_dp), bad.ctypes.data_as(_ip))
        return g, bad.astype(bool)

    def residual(self):
        """Per conservative component, the L2 norm over cells of W^{n+1} - W^n
        in the last step."""
        r = np.zeros(self.dim + 2)
        self._L.orc_residual(self._h, r.ctypes.data_as(_dp))
        return r

    def wall_flux(self):
        """Macroscopic flux through every wall face (increasing face index)
        in the last step, per unit area and time: [n_wall][dim + 2]
        (Section 2.5)."""
        n = self._L.orc_n_wall(self._h)
        F = np.zeros((n, self.dim + 2))
        if n:
            self._L.orc_wall_flux(self._h, F.ctypes.data_as(_dp))
        return F


# ---- pieces, for the pin tests ---------------------------------------------
def time_integrals(dt, tau):
    c = np.zeros(5)
    lib().orc_time_integrals(float(dt), float(tau), c.ctypes.data_as(_dp))
    return c


def prim_of_cons(W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    D = len(W) - 2
    p = np.zeros(D + 2)
    lib().orc_prim_of_cons(D, W.ctypes.data_as(_dp), p.ctypes.data_as(_dp))
    return p


def cons_of_prim(p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    D = len(p) - 2
    W = np.zeros(D + 2)
    lib().orc_cons_of_prim(D, p.ctypes.data_as(_dp), W.ctypes.data_as(_dp))
    return W


def reduced_eq(p, q, Pr, u):
    """H, B, H+, B+ at velocities u[n, D] for primitive p = (rho, U, lambda)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    D = len(p) - 2
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1, D))
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = u.shape[0]
    out = [np.zeros(n) for _ in range(4)]
    lib().orc_reduced_eq(D, p.ctypes.data_as(_dp), q.ctypes.data_as(_dp), float(Pr), n,
                         u.ctypes.data_as(_dp), *[o.ctypes.data_as(_dp) for o in out])
    return out


def half_merge(pl, pr, n):
    pl, pr, n = (np.ascontiguousarray(x, dtype=np.float64) for x in (pl, pr, n))
    D = len(n)
    W0 = np.zeros(D + 2)
    lib().orc_half_merge(D, pl.ctypes.data_as(_dp), pr.ctypes.data_as(_dp), n.ctypes.data_as(_dp),
                         W0.ctypes.data_as(_dp))
    return W0


def slope_of_g0(p, dW):
    p, dW = (np.ascontiguousarray(x, dtype=np.float64) for x in (p, dW))
    a = np.zeros(len(p))
    lib().orc_slope_of_g0(len(p) - 2, p.ctypes.data_as(_dp), dW.ctypes.data_as(_dp), a.ctypes.data_as(_dp))
    return a


def time_slope_of_g0(p, a):
    p = np.ascontiguousarray(p, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    A = np.zeros(len(p))
    lib().orc_time_slope_of_g0(len(p) - 2, p.ctypes.data_as(_dp), a.ctypes.data_as(_dp), A.ctypes.data_as(_dp))
    return A


def venkat(dm, dp, eps2):
    return lib().orc_venkat(float(dm), float(dp), float(eps2))


def gauss_hermite():
    """The oracle's 4-point Gauss-Hermite rule (weight e^{-x^2})."""
    x, w = np.zeros(4), np.zeros(4)
    n = lib().orc_gauss_hermite(x.ctypes.data_as(_dp), w.ctypes.data_as(_dp))
    assert n == 4
    return x, w
