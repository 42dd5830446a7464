"""ctypes wrapper of the plain-C FP64 oracle (``sale_oracle.c``).

TEST INFRASTRUCTURE: used by the tests, the smoke check and the CPU-baseline
leg of the benchmark only. The C source holds the scheme, step by step
(O1..O12 of the oracle's fixed reading of the ScalSALE SALE step: Lagrangian
phase, Eulerian rezone and advection, Sec. I-D and Table I of the paper);
this file only marshals arrays.

State arrays follow the library-wide logical layout: cells (nz, ny, nx) and
nodes (nz+1, ny+1, nx+1) in C order, i.e. x fastest.
"""
import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

OK, DONE, EINVAL, ENOMEM, ENUMERIC, ETANGLE = 0, 1, -1, -2, -4, -5

_lib = None


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("gamma", C.c_double), ("cfl", C.c_double), ("cq", C.c_double),
                ("cl", C.c_double), ("t_end", C.c_double), ("order", C.c_int32)]


def lib():
    """Load liboracle.so, building it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build_oracle()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(C.c_double)
        cfg = C.POINTER(_Config)
        L.orc_ws_create.restype = C.c_void_p
        L.orc_ws_create.argtypes = [cfg]
        L.orc_ws_destroy.restype = None
        L.orc_ws_destroy.argtypes = [C.c_void_p]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [cfg, C.c_void_p, P, P, P, P, P, P, P]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [cfg, C.c_void_p, P, P, P, P, P, P, C.c_int64,
                              C.POINTER(C.c_int64)]
        L.orc_timestep.restype = C.c_int
        L.orc_timestep.argtypes = [cfg, C.c_void_p, P, P, P, P, P, C.c_double, P]
        L.orc_totals.restype = C.c_int
        L.orc_totals.argtypes = [cfg, P, P, P, P, P, P, P]
        L.orc_init_sod.restype = C.c_int
        L.orc_init_sod.argtypes = [cfg] + [C.c_double] * 5 + [P] * 5
        L.orc_init_sedov.restype = C.c_int
        L.orc_init_sedov.argtypes = [cfg] + [C.c_double] * 3 + [P] * 5
        L.orc_init_noh.restype = C.c_int
        L.orc_init_noh.argtypes = [cfg] + [C.c_double] * 3 + [C.c_int] + [P] * 5
        L.orc_geometry.restype = C.c_int
        L.orc_geometry.argtypes = [cfg, C.c_void_p, P, P, P, P]
        L.orc_derived.restype = C.c_int
        L.orc_derived.argtypes = [cfg, C.c_void_p, P, P, P, P, P, P, P]
        L.orc_face_swept_volume.restype = C.c_double
        L.orc_face_swept_volume.argtypes = [P, C.c_double, C.c_double]
        L.orc_max_threads.restype = C.c_int
        L.orc_max_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_vanleer.restype = C.c_double
        L.orc_vanleer.argtypes = [C.c_double, C.c_double]
        L.orc_donor_value.restype = C.c_double
        L.orc_donor_value.argtypes = [C.c_double] * 4
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Grid:
    """Mesh and scheme constants of one run (defaults: gamma 1.4, CFL 0.5,
    quadratic / linear viscosity coefficients 1.0 / 0.5, first-order remap)."""
    nx: int
    ny: int
    nz: int
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    gamma: float = 1.4
    cfl: float = 0.5
    cq: float = 1.0
    cl: float = 0.5
    t_end: float = 1.0
    order: int = 1

    def c(self):
        return _Config(self.nx, self.ny, self.nz, (C.c_double * 3)(*self.lo),
                       (C.c_double * 3)(*self.hi), self.gamma, self.cfl, self.cq, self.cl,
                       self.t_end, self.order)

    @property
    def cell_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def node_shape(self):
        return (self.nz + 1, self.ny + 1, self.nx + 1)

    @property
    def spacing(self):
        return tuple((self.hi[a] - self.lo[a]) / n for a, n in enumerate((self.nx, self.ny, self.nz)))


@dataclass
class State:
    rho: np.ndarray
    e: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    t: float = 0.0
    step: int = 0

    def copy(self):
        return State(self.rho.copy(), self.e.copy(), self.u.copy(), self.v.copy(), self.w.copy(),
                     self.t, self.step)

    def fields(self):
        return {"rho": self.rho, "e": self.e, "u": self.u, "v": self.v, "w": self.w}


def empty_state(g: Grid) -> State:
    z = lambda s: np.zeros(s, dtype=np.float64)
    return State(z(g.cell_shape), z(g.cell_shape), z(g.node_shape), z(g.node_shape), z(g.node_shape))


def sod(g: Grid, x_split=0.5, rhoL=1.0, pL=1.0, rhoR=0.125, pR=0.1) -> State:
    s = empty_state(g)
    rc = lib().orc_init_sod(C.byref(g.c()), x_split, rhoL, pL, rhoR, pR, _ptr(s.rho), _ptr(s.e),
                            _ptr(s.u), _ptr(s.v), _ptr(s.w))
    if rc != OK:
        raise ValueError(f"orc_init_sod: {rc}")
    return s


def sedov(g: Grid, rho0=1.0, p0=1e-6, edep=0.125) -> State:
    s = empty_state(g)
    rc = lib().orc_init_sedov(C.byref(g.c()), rho0, p0, edep, _ptr(s.rho), _ptr(s.e), _ptr(s.u),
                              _ptr(s.v), _ptr(s.w))
    if rc != OK:
        raise ValueError(f"orc_init_sedov: {rc}")
    return s


def noh(g: Grid, rho0=1.0, p0=0.0, u0=1.0, dims=3) -> State:
    s = empty_state(g)
    rc = lib().orc_init_noh(C.byref(g.c()), rho0, p0, u0, dims, _ptr(s.rho), _ptr(s.e), _ptr(s.u),
                            _ptr(s.v), _ptr(s.w))
    if rc != OK:
        raise ValueError(f"orc_init_noh: {rc}")
    return s


class Oracle:
    """Holds the C workspace of one grid; steps a State in place."""

    def __init__(self, g: Grid):
        self.g = g
        self._cfg = g.c()
        self._ws = lib().orc_ws_create(C.byref(self._cfg))
        if not self._ws:
            raise MemoryError("orc_ws_create failed")

    def close(self):
        if self._ws:
            lib().orc_ws_destroy(self._ws)
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s: State):
        for a, shp in ((s.rho, self.g.cell_shape), (s.e, self.g.cell_shape), (s.u, self.g.node_shape),
                       (s.v, self.g.node_shape), (s.w, self.g.node_shape)):
            if a.shape != shp or a.dtype != np.float64 or not a.flags.c_contiguous:
                raise ValueError("state arrays do not match the grid")

    def step(self, s: State):
        """One step in place. Returns (code, dt)."""
        self._check(s)
        t = C.c_double(s.t)
        dt = C.c_double(0.0)
        rc = lib().orc_step(C.byref(self._cfg), self._ws, _ptr(s.rho), _ptr(s.e), _ptr(s.u),
                            _ptr(s.v), _ptr(s.w), C.byref(t), C.byref(dt))
        if rc == OK:
            s.t = t.value
            s.step += 1
        return rc, dt.value

    def run(self, s: State, max_steps: int = 1 << 40):
        """Steps until t >= t_end or max_steps; returns (code, steps taken)."""
        self._check(s)
        t = C.c_double(s.t)
        n = C.c_int64(0)
        rc = lib().orc_run(C.byref(self._cfg), self._ws, _ptr(s.rho), _ptr(s.e), _ptr(s.u),
                           _ptr(s.v), _ptr(s.w), C.byref(t), max_steps, C.byref(n))
        s.t = t.value
        s.step += n.value
        return rc, n.value

    def timestep(self, s: State):
        self._check(s)
        dt = C.c_double(0.0)
        rc = lib().orc_timestep(C.byref(self._cfg), self._ws, _ptr(s.rho), _ptr(s.e), _ptr(s.u),
                                _ptr(s.v), _ptr(s.w), s.t, C.byref(dt))
        return rc, dt.value

    def lagrangian_volumes(self, dX, dY, dZ):
        """Cell volumes after moving the nodes by (dX, dY, dZ) (O8 alone)."""
        VL = np.zeros(self.g.cell_shape)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (dX, dY, dZ)]
        rc = lib().orc_geometry(C.byref(self._cfg), self._ws, *(_ptr(a) for a in arrs), _ptr(VL))
        return rc, VL

    def derived(self, s: State):
        """(p, q) of a state."""
        self._check(s)
        p = np.zeros(self.g.cell_shape)
        q = np.zeros(self.g.cell_shape)
        rc = lib().orc_derived(C.byref(self._cfg), self._ws, _ptr(s.rho), _ptr(s.e), _ptr(s.u), _ptr(s.v),
                               _ptr(s.w), _ptr(p), _ptr(q))
        if rc != OK:
            raise ValueError(f"orc_derived: {rc}")
        return p, q

    def totals(self, s: State):
        """(total mass, total energy) of a state."""
        self._check(s)
        m = C.c_double(0.0)
        E = C.c_double(0.0)
        rc = lib().orc_totals(C.byref(self._cfg), _ptr(s.rho), _ptr(s.e), _ptr(s.u), _ptr(s.v),
                              _ptr(s.w), C.byref(m), C.byref(E))
        if rc != OK:
            raise ValueError(f"orc_totals: {rc}")
        return m.value, E.value


def max_threads() -> int:
    """OpenMP threads of the oracle's loops in this process."""
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of this thread's later oracle loops."""
    lib().orc_set_threads(int(n))


def face_swept_volume(d, h1, h2):
    """Exact swept volume of one face (see the C source): d is (4, 3) with
    corners (s,t) = (0,0), (1,0), (0,1), (1,1) and components (normal, t1, t2)."""
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(4, 3)
    return lib().orc_face_swept_volume(_ptr(d), h1, h2)


def vanleer(a_minus, a_plus):
    """The oracle's slope limiter (second-order remap)."""
    return lib().orc_vanleer(a_minus, a_plus)


def donor_value(q, slope, h, dvA):
    """The oracle's donor value at a swept volume's centroid (second-order
    remap): dvA is the swept volume over the face area, signed."""
    return lib().orc_donor_value(q, slope, h, dvA)
