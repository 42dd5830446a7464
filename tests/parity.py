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


def local_errors(gpu: dict, ora: "orc.State", prev: "orc.State" = None, floor=None):
    """Errors measured cell by cell (node by node), beside the max-normalised
    metric above, which on a blast checks mainly the hottest cells:

    - ``local``: max |g - o| / max(|o|, floor) per field (velocity
      components: against max(speed of the node, floor)), and its 99.9%
      quantile ``local_q999``;
    - ``l1``: sum |g - o| / sum |o| over the cells / nodes whose oracle value
      the step changed (all of them without ``prev``), for velocity over the
      three components together.

    ``floor`` maps a field to the value below which it is measured absolutely
    (default: 1e-12 of the field's largest magnitude)."""
    floor = dict(floor or {})
    out = {"local": {}, "local_q999": {}, "l1": {}}
    spd = np.sqrt(ora.u ** 2 + ora.v ** 2 + ora.w ** 2)
    vmax = float(spd.max())
    for k in FIELDS:
        g, o = np.asarray(gpu[k], dtype=np.float64), getattr(ora, k)
        d = np.abs(g - o)
        if k in ("rho", "e"):
            fl = floor.get(k, 1e-12 * float(np.abs(o).max()))
            ref = np.maximum(np.abs(o), fl)
        else:
            fl = floor.get("u", 1e-12 * vmax)
            ref = np.maximum(spd, fl)
        if fl == 0.0 and not np.all(ref > 0):
            ref = np.where(ref > 0, ref, 1e-300)
        r = d / ref
        out["local"][k] = float(r.max()) if r.size else 0.0
        out["local_q999"][k] = float(np.quantile(r, 0.999)) if r.size else 0.0
    for grp in (("rho",), ("e",), ("u", "v", "w")):
        num = den = 0.0
        for k in grp:
            g, o = np.asarray(gpu[k], dtype=np.float64), getattr(ora, k)
            m = np.ones(o.shape, dtype=bool) if prev is None else (o != getattr(prev, k))
            num += float(np.abs(g - o)[m].sum())
            den += float(np.abs(o)[m].sum())
        out["l1"]["u" if len(grp) == 3 else grp[0]] = num / den if den > 0 else (0.0 if num == 0 else np.inf)
    return out


def grid_of(cfg) -> "orc.Grid":
    return orc.Grid(cfg.nx, cfg.ny, cfg.nz, lo=tuple(cfg.lo), hi=tuple(cfg.hi), gamma=cfg.gamma,
                    cfl=cfg.cfl, cq=cfg.c_quad, cl=cfg.c_lin, t_end=cfg.t_end,
                    order=2 if cfg.remap_order == 2 else 1)


def oracle_state(fields: dict, t=0.0, step=0) -> "orc.State":
    return orc.State(*(np.ascontiguousarray(fields[k], dtype=np.float64).copy() for k in FIELDS), t=t,
                     step=step)
