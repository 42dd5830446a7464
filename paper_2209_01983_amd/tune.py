"""Autotuner of the step kernels' launch shape.

The two z-marching step kernels take a tile shape (36 x rows columns, rows 7,
14 or 28, chosen per kernel) and a target block count for the split of the z
extent into segments. Results do not depend on the shape; speed does, per
mesh size and precision. `tune` times every candidate with the library's
per-kernel event timing on a live run and keeps the fastest; results are
cached in a JSON file keyed by (GPU architecture, kernel, nx, ny, nz,
precision, remap order, mode, digest of the kernel sources), so an entry
dies with the kernels it was timed on. The second-order remap's passes have
a fixed shape, so for remap order 2 only the Lagrange kernel's rows are
tuned. `apply` sets a run's shape from the cache (tuning on a miss if asked
to).
"""
import hashlib
import json
import os

from . import sale

ROWS = (7, 14, 28)
TARGETS = (0, 1024, 2048, 3072, 6144, 12288)  # 0: the library's automatic split
KERNELS = ("lagrange", "remap")


def cache_path():
    return os.environ.get("SALE_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "sale",
                                                             "launch.json")


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


_DIGEST = None


def source_digest():
    """Digest of the library's kernel sources (the tile shapes' timings are
    only as good as the kernels they were measured on)."""
    global _DIGEST
    if _DIGEST is None:
        h = hashlib.sha256()
        d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
        for f in sorted(os.listdir(d)):
            if f.endswith((".h", ".hip")):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(f.encode() + b"\0" + fh.read())
        _DIGEST = h.hexdigest()[:16]
    return _DIGEST


def key(gpu_arch, kernel, cfg):
    prec = "fp64" if cfg.precision == sale.SALE_FP64 else "mixed32"
    order = 2 if cfg.remap_order == 2 else 1
    mode = "lagrangian" if cfg.mode == sale.SALE_LAGRANGIAN else "eulerian"
    return f"{gpu_arch}|{kernel}|{cfg.nx}x{cfg.ny}x{cfg.nz}|{prec}|order{order}|{mode}|{source_digest()}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(times):
    """times[(rows, target)] = (ms Lagrange, ms remap) -> the shape with the
    smallest step time: one shared target, the best rows per kernel for it."""
    best = None
    for t in sorted({t for _, t in times}):
        ra = min((r for r, tt in times if tt == t), key=lambda r: times[(r, t)][0])
        rb = min((r for r, tt in times if tt == t), key=lambda r: times[(r, t)][1])
        ms = times[(ra, t)][0] + times[(rb, t)][1]
        if best is None or ms < best["ms"]:
            best = {"rows_a": ra, "rows_b": rb, "target": t, "ms": ms,
                    "ms_a": times[(ra, t)][0], "ms_b": times[(rb, t)][1]}
    return best


def tune(cfg, prob=None, steps=6, warmup=2, rows=ROWS, targets=TARGETS, path=None, save=True):
    """Time every candidate shape on a run of `cfg` (Sedov by default) and
    return the chosen shape (also written to the cache)."""
    run = sale.SaleRun(cfg, prob or sale.sedov_problem())
    times = {}
    order2 = cfg.remap_order == 2
    for t in targets:
        for r in rows:
            # (order 2: the remap passes ignore the remap rows; keep them at 14)
            run.set_launch(r, 14 if order2 else r, t)
            run.step(warmup)
            ms = run.step_timed(steps)
            times[(r, t)] = (ms[1] / steps, ms[2] / steps)
    run.close()
    best = choose(times)
    if order2:
        best["rows_b"] = 14
    if save:
        cache = load_cache(path)
        a = arch()
        cache[key(a, "lagrange", cfg)] = {"rows": best["rows_a"], "target": best["target"], "ms": best["ms_a"]}
        cache[key(a, "remap", cfg)] = {"rows": best["rows_b"], "target": best["target"], "ms": best["ms_b"]}
        save_cache(cache, path)
    best["candidates"] = {f"{r}x{t}": v for (r, t), v in times.items()}
    return best


def lookup(cfg, path=None):
    cache = load_cache(path)
    a = arch()
    ea, eb = cache.get(key(a, "lagrange", cfg)), cache.get(key(a, "remap", cfg))
    if not ea or not eb:
        return None
    return {"rows_a": ea["rows"], "rows_b": eb["rows"], "target": ea["target"]}


def apply(run, tune_on_miss=False, path=None):
    """Set `run`'s launch shape from the cache; returns the shape or None."""
    shape = lookup(run.cfg, path)
    if shape is None and tune_on_miss:
        shape = tune(run.cfg, path=path)
    if shape is not None:
        run.set_launch(shape["rows_a"], shape["rows_b"], shape["target"])
    return shape
