"""Seeded synthetic inputs shared by the tests, the benchmark and the
oracle-side checks. Holds random draws only -- none of the scheme's
arithmetic -- so that neither side of a parity test depends on the other.

Arrays follow the library's logical layout: cells (nz, ny, nx), nodes
(nz+1, ny+1, nx+1), x fastest, float64.
"""
import math

import numpy as np

# Seeds of the two multi-run workloads.
BATCH_SEED = 2209
SERVE_SEED = 1983


def random_state(nx, ny, nz, seed, *, rho=(0.5, 2.0), e=(0.5, 3.0), vel=0.3, smooth=False):
    """A random admissible state: positive density and internal energy,
    node velocities with zero wall-normal components (reflective walls).

    smooth=False draws independent values per cell/node (exercises every
    branch); smooth=True draws a few random low-frequency modes."""
    rng = np.random.default_rng(seed)
    cs, ns = (nz, ny, nx), (nz + 1, ny + 1, nx + 1)
    if smooth:
        def field(shape, lo, hi):
            z, y, x = np.meshgrid(*[np.linspace(0, 1, s) for s in shape], indexing="ij")
            f = np.zeros(shape)
            for _ in range(3):
                kx, ky, kz = rng.integers(0, 3, size=3)
                ph = rng.uniform(0, 2 * math.pi, size=3)
                f += (np.cos(math.pi * kx * x + ph[0]) * np.cos(math.pi * ky * y + ph[1])
                      * np.cos(math.pi * kz * z + ph[2]))
            f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
            return lo + (hi - lo) * f
        r = field(cs, *rho)
        ee = field(cs, *e)
        u = field(ns, -vel, vel)
        v = field(ns, -vel, vel)
        w = field(ns, -vel, vel)
    else:
        r = rng.uniform(*rho, size=cs)
        ee = rng.uniform(*e, size=cs)
        u = rng.uniform(-vel, vel, size=ns)
        v = rng.uniform(-vel, vel, size=ns)
        w = rng.uniform(-vel, vel, size=ns)
    u[:, :, 0] = 0.0
    u[:, :, -1] = 0.0
    v[:, 0, :] = 0.0
    v[:, -1, :] = 0.0
    w[0, :, :] = 0.0
    w[-1, :, :] = 0.0
    return {"rho": r, "e": ee, "u": u, "v": v, "w": w}


def batch_mix(n_runs=256, seed=BATCH_SEED, edge=(16, 64)):
    """Parameters of the batched workload: per run (kind, nx, ny, nz, params).
    The first half are Sod tubes (density ratio U[4,16], pressure ratio
    U[5,20]); the second half Sedov blasts (deposited energy U[0.05, 1.0])."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(n_runs):
        nx, ny, nz = (int(a) for a in rng.integers(edge[0], edge[1] + 1, size=3))
        if r < n_runs // 2:
            runs.append({"kind": "sod", "n": (nx, ny, nz), "rho_ratio": float(rng.uniform(4, 16)),
                         "p_ratio": float(rng.uniform(5, 20))})
        else:
            runs.append({"kind": "sedov", "n": (nx, ny, nz), "edep": float(rng.uniform(0.05, 1.0))})
    return runs


def serve_trace(n_requests=1000, seed=SERVE_SEED, rate=50.0, edge=(32, 192), steps=(100, 500)):
    """Poisson arrival trace of the serving workload: arrival time (s), cubic
    edge drawn log-uniformly, step count, and a 50/50 Sod/Sedov mix with the
    same parameter ranges as the batched workload."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for a in range(n_requests):
        n = int(round(math.exp(rng.uniform(math.log(edge[0]), math.log(edge[1])))))
        ns = int(rng.integers(steps[0], steps[1] + 1))
        if rng.uniform() < 0.5:
            out.append({"arrival": float(t[a]), "kind": "sod", "n": (n, n, n), "steps": ns,
                        "rho_ratio": float(rng.uniform(4, 16)), "p_ratio": float(rng.uniform(5, 20))})
        else:
            out.append({"arrival": float(t[a]), "kind": "sedov", "n": (n, n, n), "steps": ns,
                        "edep": float(rng.uniform(0.05, 1.0))})
    return out
