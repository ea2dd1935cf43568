"""ctypes binding of libugks.so (include/ugks.h): argument marshalling only.

Every step of the scheme runs in the HIP library; this module converts numpy
arrays into the C structs, passes torch's current HIP stream, and turns
status codes into exceptions.  It raises at import of the library when the
built libugks.so is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugks.so")

UGKS_OK, UGKS_ERR_ARG, UGKS_ERR_ALLOC, UGKS_ERR_HIP, UGKS_ERR_NONPHYSICAL, UGKS_ERR_STATE = 0, -1, -2, -3, -4, -5
UGKS_F64, UGKS_F32, UGKS_BF16 = 0, 1, 2
UGKS_BC_INTERIOR, UGKS_BC_INFLOW, UGKS_BC_OUTFLOW, UGKS_BC_WALL = 0, 1, 2, 3
_FSTORE = {"f64": UGKS_F64, "f32": UGKS_F32, "bf16": UGKS_BF16}
UGKS_MEM_TWO_BUFFERS, UGKS_MEM_IN_PLACE = 0, 1
_MEM = {"two-buffers": UGKS_MEM_TWO_BUFFERS, "in-place": UGKS_MEM_IN_PLACE}
UGKS_DEFAULT_CHUNK = 1024
UGKS_STATIC_BATCH_MAX = 64
UGKS_SWEEP_AUTO, UGKS_SWEEP_GATHER, UGKS_SWEEP_PUSH, UGKS_SWEEP_PUSH_UNORDERED = 0, 1, 2, 3
_SWEEP = {"auto": UGKS_SWEEP_AUTO, "gather": UGKS_SWEEP_GATHER, "push": UGKS_SWEEP_PUSH,
          "push_unordered": UGKS_SWEEP_PUSH_UNORDERED}
_ERRNAMES = {-1: "UGKS_ERR_ARG", -2: "UGKS_ERR_ALLOC", -3: "UGKS_ERR_HIP", -4: "UGKS_ERR_NONPHYSICAL",
             -5: "UGKS_ERR_STATE"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class ugks_mesh_t(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_cells", C.c_int), ("n_faces", C.c_int),
                ("cell_volume", _dp), ("cell_centroid", _dp), ("face_cells", _ip),
                ("face_normal", _dp), ("face_area", _dp), ("face_centroid", _dp), ("face_shift", _dp),
                ("face_bc", _ip), ("face_bc_id", _ip)]


class ugks_vgrid_t(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_vel", C.c_int), ("u", _dp), ("w", _dp)]


class ugks_gas_t(C.Structure):
    _fields_ = [("Pr", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double), ("cfl", C.c_double),
                ("dt_override", C.c_double), ("limiter_k", C.c_double), ("limiter", C.c_int),
                ("fstore", C.c_int), ("n_bc", C.c_int), ("bc_prim", _dp), ("mem_mode", C.c_int),
                ("chunk", C.c_int), ("sweep", C.c_int)]


class UgksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libugks.so and declare the C ABI.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run paper_2412_06546_amd/build.py (or __graft_entry__.build())")
    # PyTorch ships its own HIP runtime.  Loaded first, it is the runtime the
    # library binds to (same soname); loaded after the library, a second HIP
    # and HSA runtime would enter the process and the two would not share
    # devices, memory or streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    L.ugks_create.restype = C.c_int
    L.ugks_create.argtypes = [C.POINTER(ugks_mesh_t), C.POINTER(ugks_vgrid_t), C.POINTER(ugks_gas_t), _dp,
                              C.c_void_p, C.POINTER(C.c_void_p)]
    L.ugks_step.restype = C.c_int
    L.ugks_step.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ugks_step_async.restype = C.c_int
    L.ugks_step_async.argtypes = [C.c_void_p, C.c_int]
    L.ugks_poll.restype = C.c_int
    L.ugks_poll.argtypes = [C.c_void_p, C.POINTER(C.c_int), _dp]
    L.ugks_footprint_estimate.restype = C.c_size_t
    L.ugks_footprint_estimate.argtypes = [C.POINTER(ugks_mesh_t), C.POINTER(ugks_vgrid_t), C.POINTER(ugks_gas_t)]
    L.ugks_macros.restype = C.c_int
    L.ugks_macros.argtypes = [C.c_void_p, _dp, _dp]
    L.ugks_get_f.restype = C.c_int
    L.ugks_get_f.argtypes = [C.c_void_p, _dp]
    L.ugks_set_f.restype = C.c_int
    L.ugks_set_f.argtypes = [C.c_void_p, _dp]
    L.ugks_dt.restype = C.c_double
    L.ugks_dt.argtypes = [C.c_void_p]
    L.ugks_n_comp.restype = C.c_int
    L.ugks_n_comp.argtypes = [C.c_void_p]
    L.ugks_step_count.restype = C.c_long
    L.ugks_step_count.argtypes = [C.c_void_p]
    L.ugks_footprint_bytes.restype = C.c_size_t
    L.ugks_footprint_bytes.argtypes = [C.c_void_p]
    L.ugks_sweep_kind.restype = C.c_int
    L.ugks_sweep_kind.argtypes = [C.c_void_p]
    L.ugks_sweep_colours.restype = C.c_int
    L.ugks_sweep_colours.argtypes = [C.c_void_p]
    L.ugks_is_tensor_grid.restype = C.c_int
    L.ugks_is_tensor_grid.argtypes = [C.c_void_p]
    L.ugks_profile.restype = C.c_int
    L.ugks_profile.argtypes = [C.c_void_p, C.c_int]
    L.ugks_profile_read.restype = C.c_int
    L.ugks_profile_read.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_long)]
    L.ugks_velocity_order.restype = C.c_int
    L.ugks_velocity_order.argtypes = [C.c_void_p, _ip]
    L.ugks_state_bytes.restype = C.c_size_t
    L.ugks_state_bytes.argtypes = [C.c_void_p]
    L.ugks_get_state.restype = C.c_int
    L.ugks_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.ugks_set_state.restype = C.c_int
    L.ugks_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.ugks_n_wall_faces.restype = C.c_int
    L.ugks_n_wall_faces.argtypes = [C.c_void_p]
    L.ugks_wall_flux.restype = C.c_int
    L.ugks_wall_flux.argtypes = [C.c_void_p, _dp]
    L.ugks_surface.restype = C.c_int
    L.ugks_surface.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp]
    L.ugks_cell_order.restype = C.c_int
    L.ugks_cell_order.argtypes = [C.c_void_p, _ip]
    L.ugks_device_f.restype = C.c_void_p
    L.ugks_device_f.argtypes = [C.c_void_p]
    L.ugks_batch_create.restype = C.c_int
    L.ugks_batch_create.argtypes = [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
    L.ugks_batch_step.restype = C.c_int
    L.ugks_batch_step.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int]
    L.ugks_batch_last_error.restype = C.c_char_p
    L.ugks_batch_last_error.argtypes = [C.c_void_p]
    L.ugks_batch_step_static.restype = C.c_int
    L.ugks_batch_step_static.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p]
    L.ugks_batch_destroy.restype = None
    L.ugks_batch_destroy.argtypes = [C.c_void_p]
    L.ugks_destroy.restype = None
    L.ugks_destroy.argtypes = [C.c_void_p]
    L.ugks_last_error.restype = C.c_char_p
    L.ugks_last_error.argtypes = [C.c_void_p]
    _lib = L
    return L


def _check(L, h, code):
    if code != UGKS_OK:
        raise UgksError(code, L.ugks_last_error(h).decode())


def current_stream_handle():
    """torch's current HIP stream as a hipStream_t (None = default stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


def _structs(case, fstore, keep, mem="two-buffers", chunk=0, sweep="auto"):
    """ugks_mesh_t, ugks_vgrid_t, ugks_gas_t and prim0 for a case dict; the
    numpy buffers they point to are appended to keep."""
    m, vg, gas = case["mesh"], case["vgrid"], case["gas"]
    dim = int(m["dim"])

    def d(x):
        a = np.ascontiguousarray(x, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(_dp)

    def i(x):
        a = np.ascontiguousarray(x, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(_ip)

    mesh = ugks_mesh_t(dim, len(m["cell_volume"]), len(m["face_area"]), d(m["cell_volume"]), d(m["cell_centroid"]),
                       i(m["face_cells"]), d(m["face_normal"]), d(m["face_area"]), d(m["face_centroid"]),
                       d(m["face_shift"]) if m.get("face_shift") is not None else None,
                       i(m["face_bc"]), i(m["face_bc_id"]))
    vgrid = ugks_vgrid_t(dim, len(vg["w"]), d(vg["u"]), d(vg["w"]))
    bc = np.asarray(gas["bc_prim"], dtype=np.float64)
    g = ugks_gas_t(gas["Pr"], gas["omega"], gas["mu_ref"], gas["cfl"], gas["dt_override"], gas["limiter_k"],
                   int(gas["limiter"]), _FSTORE[fstore], bc.shape[0], d(bc), _MEM[mem], int(chunk), _SWEEP[sweep])
    return mesh, vgrid, g, d(case["prim0"])


def footprint_estimate(case, fstore: str = "f64", mem: str = "two-buffers", chunk: int = 0,
                       sweep: str = "auto") -> int:
    """Device bytes ugks_create would allocate for this case (host only)."""
    L = load_library()
    keep = []
    mesh, vgrid, g, _ = _structs(case, fstore, keep, mem, chunk, sweep)
    return int(L.ugks_footprint_estimate(C.byref(mesh), C.byref(vgrid), C.byref(g)))


class Solver:
    """A flow case on the GPU: ugks_create ... ugks_destroy."""

    def __init__(self, case, fstore: str = "f64", stream=None, mem: str = "two-buffers", chunk: int = 0,
                 sweep: str = "auto"):
        """mem: 'two-buffers' (f^n and f^{n+1} in separate buffers) or
        'in-place' (one f buffer plus a ring of `chunk` velocities per cell);
        sweep: 'auto', 'gather', 'push' or 'push_unordered' (UGKS_SWEEP_*)."""
        L = self._L = load_library()
        self.dim = int(case["mesh"]["dim"])
        self.nc = len(case["mesh"]["cell_volume"])
        self.nv = len(case["vgrid"]["w"])
        keep = []
        mesh, vgrid, g, prim0 = _structs(case, fstore, keep, mem, chunk, sweep)
        if stream is None:
            stream = current_stream_handle()
        self.stream = stream
        h = C.c_void_p()
        code = L.ugks_create(C.byref(mesh), C.byref(vgrid), C.byref(g), prim0, stream, C.byref(h))
        _check(L, None, code)
        self._h = h
        self.ncomp = L.ugks_n_comp(h)

    def close(self):
        if getattr(self, "_h", None):
            self._L.ugks_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    @property
    def dt(self) -> float:
        return self._L.ugks_dt(self._h)

    @property
    def step_count(self) -> int:
        return self._L.ugks_step_count(self._h)

    @property
    def footprint_bytes(self) -> int:
        return self._L.ugks_footprint_bytes(self._h)

    @property
    def sweep(self) -> str:
        """'push', 'push_unordered' or 'gather': how this handle's steps evaluate the face fluxes."""
        return {UGKS_SWEEP_PUSH: "push", UGKS_SWEEP_PUSH_UNORDERED: "push_unordered",
                UGKS_SWEEP_GATHER: "gather"}[self._L.ugks_sweep_kind(self._h)]

    @property
    def n_colours(self) -> int:
        """Colour classes of the push sweep (one launch each per step); 0 when gathering."""
        return self._L.ugks_sweep_colours(self._h)

    @property
    def tensor_grid(self) -> bool:
        return bool(self._L.ugks_is_tensor_grid(self._h))

    def step(self, n: int = 1, residual: bool = False):
        r = np.zeros(self.dim + 2) if residual else None
        _check(self._L, self._h, self._L.ugks_step(self._h, int(n), r.ctypes.data_as(_dp) if residual else None))
        return r

    def step_async(self, n: int = 1):
        """Enqueue n steps and return at once (see poll)."""
        _check(self._L, self._h, self._L.ugks_step_async(self._h, int(n)))

    def poll(self):
        """None while the enqueued steps run, else the last step's residual."""
        done = C.c_int(0)
        r = np.zeros(self.dim + 2)
        _check(self._L, self._h, self._L.ugks_poll(self._h, C.byref(done), r.ctypes.data_as(_dp)))
        return r if done.value else None

    def macros(self):
        W = np.zeros((self.nc, self.dim + 2))
        q = np.zeros((self.nc, self.dim))
        _check(self._L, self._h, self._L.ugks_macros(self._h, W.ctypes.data_as(_dp), q.ctypes.data_as(_dp)))
        return W, q

    def f(self):
        f = np.zeros((self.nc, self.ncomp, self.nv))
        _check(self._L, self._h, self._L.ugks_get_f(self._h, f.ctypes.data_as(_dp)))
        return f

    def velocity_order(self):
        """Stored velocity position -> caller's velocity index."""
        perm = np.zeros(self.nv, dtype=np.int32)
        _check(self._L, self._h, self._L.ugks_velocity_order(self._h, perm.ctypes.data_as(_ip)))
        return perm

    def get_state(self) -> bytes:
        """Exact checkpoint (W, q, f in storage precision, step count)."""
        n = self._L.ugks_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        _check(self._L, self._h, self._L.ugks_get_state(self._h, buf, n))
        return buf.raw

    def set_state(self, state: bytes):
        """Restore a checkpoint taken from a solver of the same case."""
        buf = C.create_string_buffer(bytes(state), len(state))
        _check(self._L, self._h, self._L.ugks_set_state(self._h, buf, len(state)))

    def wall_flux(self):
        """Macroscopic flux through every wall face in the last step, per unit
        area and time: [n_wall][dim + 2] (mass, momentum, energy)."""
        n = self._L.ugks_n_wall_faces(self._h)
        F = np.zeros((n, self.dim + 2))
        _check(self._L, self._h, self._L.ugks_wall_flux(self._h, F.ctypes.data_as(_dp)))
        return F

    def surface(self, rho_inf: float, u_inf: float):
        """Surface pressure, shear stress and heat flux of every wall face in
        the last step and the coefficients Cp, Ct, Ch (ugks_surface)."""
        n = self._L.ugks_n_wall_faces(self._h)
        out = np.zeros((n, 6))
        _check(self._L, self._h, self._L.ugks_surface(self._h, float(rho_inf), float(u_inf),
                                                      out.ctypes.data_as(_dp)))
        return {"p": out[:, 0], "sigma": out[:, 1], "q": out[:, 2], "Cp": out[:, 3], "Ct": out[:, 4],
                "Ch": out[:, 5]}

    def cell_order(self):
        """Stored cell position -> caller's cell index."""
        perm = np.zeros(self.nc, dtype=np.int32)
        _check(self._L, self._h, self._L.ugks_cell_order(self._h, perm.ctypes.data_as(_ip)))
        return perm

    def profile(self, enable: bool = True):
        _check(self._L, self._h, self._L.ugks_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(ms in the sweep kernel, ms in the prologue kernels, steps timed)."""
        ms = np.zeros(2)
        n = C.c_long(0)
        _check(self._L, self._h, self._L.ugks_profile_read(self._h, ms.ctypes.data_as(_dp), C.byref(n)))
        return float(ms[0]), float(ms[1]), int(n.value)

    def set_f(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64)
        assert a.shape == (self.nc, self.ncomp, self.nv)
        _check(self._L, self._h, self._L.ugks_set_f(self._h, a.ctypes.data_as(_dp)))


class Batch:
    """Several cases advanced by the same launches (ugks_batch_*).  Every
    Solver passed to step() must have been created on the batch's stream."""

    def __init__(self, max_cases: int, stream=None):
        L = self._L = load_library()
        if stream is None:
            stream = current_stream_handle()
        self.stream = stream
        h = C.c_void_p()
        code = L.ugks_batch_create(int(max_cases), stream, C.byref(h))
        if code != UGKS_OK:
            raise UgksError(code, L.ugks_batch_last_error(None).decode())
        self._h = h
        self.max_cases = int(max_cases)

    def step(self, solvers, nsteps: int):
        """Enqueue nsteps steps of every solver; each is then pending (poll)."""
        arr = (C.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
        code = self._L.ugks_batch_step(self._h, arr, len(solvers), int(nsteps))
        if code != UGKS_OK:
            raise UgksError(code, self._L.ugks_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.ugks_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def batch_step_static(solvers, nsteps: int, stream=None):
    """ugks_batch_step_static: the batched step without a batch object (no
    allocation); every solver must have been created on `stream`."""
    L = load_library()
    if stream is None:
        stream = current_stream_handle()
    arr = (C.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
    code = L.ugks_batch_step_static(arr, len(solvers), int(nsteps), stream)
    if code != UGKS_OK:
        raise UgksError(code, L.ugks_batch_last_error(None).decode())
