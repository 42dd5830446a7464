"""Helpers of the GPU parity tests (not collected by pytest).

The parity metric of a field f: max |f_gpu - f_oracle| / scale, where the
scale of rho and e is max |f_oracle| and the scale of each velocity
component is the largest oracle speed component over u, v and w (velocity is
one vector field: a component that is pure rounding noise, like the
transverse velocity of the Sod tube, is measured against the flow's speed,
not against its own noise). A field the oracle has identically zero (scale
0) must be zero on the GPU too. FP64 bar: 1e-12 per field per step.
"""
import sys

import numpy as np

from oracle import oracle as orc

FIELDS = ("rho", "e", "u", "v", "w")
TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field_error(g, o):
    scale = np.abs(o).max() if o.size else 0.0
    if scale == 0.0:
        return 0.0 if np.all(g == 0.0) else np.inf
    return float(np.abs(g - o).max() / max(scale, 1e-300))


def field_error_scaled(g, o, scale):
    if scale == 0.0:
        return 0.0 if np.all(g == 0.0) else np.inf
    return float(np.abs(g - o).max() / scale)


def errors(gpu: dict, ora: "orc.State"):
    vs = max(np.abs(ora.u).max(), np.abs(ora.v).max(), np.abs(ora.w).max())
    out = {k: field_error(gpu[k], getattr(ora, k)) for k in ("rho", "e")}
    for k in ("u", "v", "w"):
        out[k] = field_error_scaled(gpu[k], getattr(ora, k), vs)
    return out


def assert_parity(gpu, ora, tol=TOL64, what=""):
    err = errors(gpu, ora)
    bad = {k: v for k, v in err.items() if not v <= tol}
    assert not bad, f"{what}: {bad}"
    return err


def grid_of(cfg) -> "orc.Grid":
    return orc.Grid(cfg.nx, cfg.ny, cfg.nz, lo=tuple(cfg.lo), hi=tuple(cfg.hi), gamma=cfg.gamma,
                    cfl=cfg.cfl, cq=cfg.c_quad, cl=cfg.c_lin, t_end=cfg.t_end,
                    order=2 if cfg.remap_order == 2 else 1)


def oracle_state(fields: dict, t=0.0, step=0) -> "orc.State":
    return orc.State(*(np.ascontiguousarray(fields[k], dtype=np.float64).copy() for k in FIELDS), t=t,
                     step=step)
