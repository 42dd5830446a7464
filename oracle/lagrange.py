"""ctypes wrapper of the pure-Lagrangian oracle step (``lagrange_oracle.c``).

TEST INFRASTRUCTURE: used by the tests only. The C source holds the scheme
(L1..L8, the oracle's reading of the paper's Lagrangian rezoning mode, Table I
and Fig. 2a); this file only marshals arrays. Layout as the Eulerian oracle:
cells (nz, ny, nx), nodes (nz+1, ny+1, nx+1), x fastest.
"""
import ctypes as C
from dataclasses import dataclass

import numpy as np

from .oracle import DONE, OK, State, lib as _lib  # noqa: F401  (codes shared with the Eulerian oracle)


class _LConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("gamma", C.c_double), ("cfl", C.c_double), ("cq", C.c_double), ("cl", C.c_double),
                ("chg", C.c_double), ("t_end", C.c_double)]


_ready = False


def lib():
    global _ready
    L = _lib()
    if not _ready:
        P = C.POINTER(C.c_double)
        cfg = C.POINTER(_LConfig)
        L.olg_hex.restype = None
        L.olg_hex.argtypes = [P, P, P]
        L.olg_length.restype = C.c_double
        L.olg_length.argtypes = [P, C.c_double]
        L.olg_cell_forces.restype = C.c_int
        L.olg_cell_forces.argtypes = [cfg, P, P, C.c_double, C.c_double, C.c_double, P]
        L.olg_timestep.restype = C.c_int
        L.olg_timestep.argtypes = [cfg] + [P] * 8 + [C.c_double, P]
        L.olg_step.restype = C.c_int
        L.olg_step.argtypes = [cfg] + [P] * 7 + [P, P, P]
        L.olg_density.restype = C.c_int
        L.olg_density.argtypes = [cfg, P, P, P, P, P]
        _ready = True
    return L


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def hex_geometry(X):
    """(corner vectors S[8,3], volume) of the trilinear hex with corners X[8,3]
    (corner a = bits (a&1, a>>1&1, a>>2&1) along x, y, z)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    S = np.zeros((8, 3))
    V = C.c_double(0.0)
    lib().olg_hex(_p(X), _p(S), C.byref(V))
    return S, V.value


def hex_length(X, V):
    X = np.ascontiguousarray(X, dtype=np.float64)
    return lib().olg_length(_p(X), V)


@dataclass
class LagGrid:
    nx: int
    ny: int
    nz: int
    gamma: float = 1.4
    cfl: float = 0.5
    cq: float = 1.0
    cl: float = 0.5
    chg: float = 0.1
    t_end: float = 1.0

    def c(self):
        return _LConfig(self.nx, self.ny, self.nz, self.gamma, self.cfl, self.cq, self.cl, self.chg, self.t_end)


def cell_forces(g: LagGrid, X, U, e, m, dt):
    F = np.zeros((8, 3))
    ok = lib().olg_cell_forces(C.byref(g.c()), _p(np.ascontiguousarray(X, dtype=np.float64)),
                               _p(np.ascontiguousarray(U, dtype=np.float64)), e, m, dt, _p(F))
    return F, bool(ok)


@dataclass
class LagState:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    e: np.ndarray
    m: np.ndarray
    t: float = 0.0
    step: int = 0

    def copy(self):
        return LagState(*(a.copy() for a in (self.x, self.y, self.z, self.u, self.v, self.w, self.e, self.m)),
                        self.t, self.step)


def from_eulerian(s: State, lo, hi) -> LagState:
    """Lagrangian state on the initial Cartesian mesh of the box [lo, hi]:
    node positions lo + (i dx, j dy, k dz), cell masses rho V0."""
    nz, ny, nx = s.rho.shape
    d = [(hi[a] - lo[a]) / n for a, n in enumerate((nx, ny, nz))]
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    x = lo[0] + I * d[0]
    y = lo[1] + J * d[1]
    z = lo[2] + K * d[2]
    V0 = d[0] * d[1] * d[2]
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64).copy()
    return LagState(f(x), f(y), f(z), f(s.u), f(s.v), f(s.w), f(s.e), f(s.rho * V0), s.t, s.step)


def density(g: LagGrid, s: LagState):
    rho = np.zeros_like(s.e)
    rc = lib().olg_density(C.byref(g.c()), _p(s.x), _p(s.y), _p(s.z), _p(s.m), _p(rho))
    if rc != OK:
        raise ValueError(rc)
    return rho


def timestep(g: LagGrid, s: LagState):
    dt = C.c_double(0.0)
    rc = lib().olg_timestep(C.byref(g.c()), _p(s.x), _p(s.y), _p(s.z), _p(s.u), _p(s.v), _p(s.w), _p(s.e),
                            _p(s.m), s.t, C.byref(dt))
    return rc, dt.value


def step(g: LagGrid, s: LagState):
    """One step in place; (code, dt)."""
    t = C.c_double(s.t)
    dt = C.c_double(0.0)
    rc = lib().olg_step(C.byref(g.c()), _p(s.x), _p(s.y), _p(s.z), _p(s.u), _p(s.v), _p(s.w), _p(s.e), _p(s.m),
                        C.byref(t), C.byref(dt))
    if rc == OK:
        s.t = t.value
        s.step += 1
    return rc, dt.value


def run(g: LagGrid, s: LagState, max_steps=1 << 40):
    n = 0
    rc = OK
    while n < max_steps:
        rc, _ = step(g, s)
        if rc != OK:
            break
        n += 1
    return rc, n


def totals(s: LagState):
    """(mass, total energy): sum m, sum m e + sum over nodes of m_p |u|^2 / 2."""
    nz, ny, nx = s.e.shape
    mp = np.zeros(s.x.shape)
    for a in range(8):
        sx, sy, sz = a & 1, (a >> 1) & 1, (a >> 2) & 1
        mp[sz:sz + nz, sy:sy + ny, sx:sx + nx] += s.m
    mp *= 0.125
    ke = 0.5 * mp * (s.u ** 2 + s.v ** 2 + s.w ** 2)
    return float(s.m.sum()), float((s.m * s.e).sum() + ke.sum())
