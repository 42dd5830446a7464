#!/usr/bin/env python3
"""Benchmark of the SALE Lagrange + remap step on one MI355X.

Headline (`value`): cell-updates/s of the FP64 step on the Sedov blast,
320^3 octant mesh of [0,1.2]^3 (rho = 1, p = 1e-6, E = 0.125 in the corner
cell, gamma 1.4, CFL 0.5), synthetic state generated on the device. W warm-up
steps, then K timed steps between HIP events on the library's stream;
value = cells x K / time. The same window in MIXED32 is reported beside it.

Also reported (one JSON line, extra keys):
  roofline     the step as the unit of the HBM roofline: algorithmic bytes =
               read + write of the state once per step, 80.45 B/cell at 320^3
               FP64, over the summed duration of the step's kernels (HIP
               events around each kernel on the library's stream); per-kernel
               durations and their compulsory bytes; HBM traffic measured
               with rocprofv3 counters when the committed counter summary
               matches the current kernel sources (else null).
  latency      Sod 64x4x4 to t = 0.2, FP64: full-run latency p50/p99 over
               repeated runs (init, steps and the status read; launch bound).
  sedov128     Sedov 128^3 to t = 1.0, FP64: full-run latency and
               cell-updates/s.
  noh128       spherical Noh implosion 128^3 to t = 0.6 (gamma 5/3, inflow
               speed 1 toward the corner, p0 = 1e-6), FP64 and MIXED32:
               full-run time, steps, cell-updates/s, peak density.
  lagrange128  pure-Lagrangian mode (the mesh moves with the flow), Sedov
               128^3, FP64: per-step throughput over a 100-step window after
               10 warm-up steps, kernel split (forces+nodes, energy+geometry).
  batched      256 runs (seeded mix of Sod / Sedov, edges 16..64), MIXED32
               and FP64, 200 steps each in ONE pool advance, in four advance
               modes (one persistent launch, the block's headline; lockstep
               kernels with the steps after the first replayed from a captured
               HIP graph; lockstep kernels all launched; no mode forced, the
               library's choice): aggregate cell-updates/s, makespan,
               per-run latency p50/p99; the same runs one after another on the
               plain FP64 path.
  serving      seeded Poisson trace (50 requests/s, cubic 32^3..192^3,
               100..500 steps), continuous batching under an HBM budget, in
               MIXED32 and FP64: throughput and arrival -> result latency.
  cpu_baseline the FP64 oracle on this host's cores, a few steps of the
               320^3 workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
KERNEL_SOURCES = ("sale_device.h", "sale_tiles.h", "sale_step.hip", "sale_impl.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_sedov320.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=320, help="cells per axis of the headline workload")
    ap.add_argument("--quick", action="store_true", help="headline and roofline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=20, help="oracle steps on all threads")
    ap.add_argument("--cpu-steps-one", type=int, default=5, help="oracle steps on one thread")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--no-tune", action="store_true", help="default launch shape, no autotuning")
    ap.add_argument("--shape", default="", metavar="A,B,T",
                    help="launch shape of the headline runs (tile rows of the two step kernels, z-split "
                         "target); skips the autotuner")
    ap.add_argument("--precision-report", type=int, default=None, metavar="N",
                    help="run the N^3 Sedov to t = 1 in FP64 and MIXED32 and report per-field errors "
                         "(default: 128 in the full run, none with --quick; 0: none)")
    ap.add_argument("--section", default="", choices=("", "latency", "sedov128", "noh128", "lagrange128", "batched", "serving"),
                    help="run only this extra block and print its JSON (for profiling it)")
    ap.add_argument("--pool-modes", default=",".join(m for m, _ in POOL_MODES),
                    help="batched block: the pool advance modes to run (comma list)")
    ap.add_argument("--batched-steps", type=int, default=200, help="batched block: steps per run")
    ap.add_argument("--batch-runs", type=int, default=256, help="batched block (--section batched): runs")
    ap.add_argument("--batch-edge", default="16,64", help="batched block (--section batched): mesh edges lo,hi")
    ap.add_argument("--no-seq", action="store_true",
                    help="batched block: skip the sequential single-run FP64 comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 2 GiB (reference for HBM counters)")
    return ap.parse_args()


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q))


# ---- byte model ------------------------------------------------------------------
def algorithmic_bytes(n, esz=8):
    """Read + write of the state once per step: rho, e per cell, u, v, w per node."""
    return 2 * (2 * n ** 3 + 3 * (n + 1) ** 3) * esz


def compulsory_bytes(n, esz=8):
    """What each step kernel must move given its inputs and outputs (R = esz
    bytes, the storage type of the state and the hand-off): Lagrange reads
    rho, e, u, v, w and writes u', v', w', e^L and the three lower-face swept
    volumes per cell; remap reads e^L, the swept volumes, rho and u', v', w'
    and writes rho, e, u, v, w."""
    c, p = n ** 3, (n + 1) ** 3
    lag = c * (2 * esz) + p * (3 * esz) + p * (3 * esz) + c * (4 * esz)
    rem = c * (4 * esz) + c * esz + p * (3 * esz) + c * (2 * esz) + p * (3 * esz)
    return {"k_lagrange": lag, "k_remap": rem}


def kernel_source_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_01983_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n, shape):
    """HBM bytes per step from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources, at this mesh size and in this
    launch shape."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel sources sha256\[:16\]:\s*([0-9a-f]{16})", text)
    b = re.search(r"traffic bytes per step \(fp64\):\s*([0-9.eE+]+)", text)
    if not m or not b:
        return None, "counter summary unreadable"
    if m.group(1) != kernel_source_digest():
        return None, "kernels changed since the counters were taken"
    w = re.search(r"counted on: (\d+)\^3, launch shape (\d+),(\d+),(\d+)", text)
    # z-split target 0 (automatic) splits a mesh this large like the target 3072
    same_split = {int(w.group(4)), shape["target"]} <= {0, 3072} if w else False
    if not w or int(w.group(1)) != n or (int(w.group(2)), int(w.group(3))) != (shape["rows_a"], shape["rows_b"]) \
            or not (int(w.group(4)) == shape["target"] or (n >= 128 and same_split)):
        return None, "counters were taken at another size or launch shape"
    return float(b.group(1)), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


# ---- workloads -----------------------------------------------------------------
def headline(n, steps, warmup, precision, tuned=True, fixed=None, order=1):
    """(ms per step from HIP events around `steps` async steps, final t,
    per-kernel ms, launch shape). With `tuned`, the autotuner first picks the
    launch shape of the step kernels for this mesh and precision."""
    import torch
    from paper_2209_01983_amd import sale, tune

    cfg = sale.make_config(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0, precision=precision, remap_order=order)
    shape = {"rows_a": 14, "rows_b": 14, "target": 0}
    if fixed:
        shape = dict(zip(("rows_a", "rows_b", "target"), fixed))
    elif tuned:
        best = tune.tune(cfg, steps=4, warmup=1, save=False)
        shape = {k: best[k] for k in ("rows_a", "rows_b", "target")}
    run = sale.SaleRun(cfg, sale.sedov_problem())
    run.set_launch(shape["rows_a"], shape["rows_b"], shape["target"])
    run.step(warmup)
    torch.cuda.synchronize()
    _, s0, _, _ = run.state()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    t1, s1, _, flags = run.state()
    if s1 - s0 != steps or flags != 0:
        raise RuntimeError(f"timed window did not run {steps} full steps ({s1 - s0}, flags {flags})")
    # per-kernel durations over a further window (events between kernels)
    kms = run.step_timed(min(steps, 50))
    nk = min(steps, 50)
    run.close()
    return ms / steps, t1, [x / nk for x in kms], shape


def sod_latency(reps):
    import torch
    from paper_2209_01983_amd import sale

    cfg = sale.make_config(64, 4, 4, hi=(1.0, 0.0625, 0.0625), t_end=0.2)
    lat, steps = [], None
    for _ in range(reps + 3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = sale.SaleRun(cfg, sale.sod_problem())
        rc = r.run()
        b = time.perf_counter()
        if rc != sale.SALE_DONE:
            raise RuntimeError(f"sod run ended with {rc}")
        steps = r.state()[1]
        r.close()
        lat.append(b - a)
    lat = lat[3:]
    return {"workload": "sod 64x4x4 to t=0.2 fp64", "runs": reps, "steps": steps,
            "p50_ms": pct(lat, 50) * 1e3, "p99_ms": pct(lat, 99) * 1e3}


def sedov128(reps):
    import torch
    from paper_2209_01983_amd import sale

    cfg = sale.make_config(128, 128, 128, hi=(1.2, 1.2, 1.2), t_end=1.0)
    lat, out = [], {}
    for k in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = sale.SaleRun(cfg, sale.sedov_problem())
        rc = r.run()
        b = time.perf_counter()
        if rc != sale.SALE_DONE:
            raise RuntimeError(f"sedov 128 run ended with {rc}")
        if k == 0:
            m1, e1 = r.totals()
            out = {"steps": r.state()[1], "mass_total": m1, "energy_total": e1}
        r.close()
        lat.append(b - a)
    steps = out["steps"]
    return {"workload": "sedov 128^3 to t=1.0 fp64", "runs": reps, "latency_s": lat,
            "p50_s": pct(lat, 50), "cell_updates_per_s": 128 ** 3 * steps / pct(lat, 50), **out}


def noh128(reps):
    import torch
    from paper_2209_01983_amd import sale

    out = {"workload": "spherical noh 128^3 of [0,1]^3 to t=0.6, gamma 5/3"}
    for name, prec in (("fp64", sale.SALE_FP64), ("mixed32", sale.SALE_MIXED32)):
        cfg = sale.make_config(128, 128, 128, gamma=5.0 / 3.0, t_end=0.6, precision=prec)
        lat, info = [], {}
        for k in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            r = sale.SaleRun(cfg, sale.noh_problem(dims=3))
            rc = r.run()
            b = time.perf_counter()
            if rc != sale.SALE_DONE:
                raise RuntimeError(f"noh 128 run ended with {rc}")
            if k == 0:
                info = {"steps": r.state()[1], "peak_rho": float(r.fields(("rho",))["rho"].max())}
            r.close()
            lat.append(b - a)
        out[name] = {"runs": reps, "p50_s": pct(lat, 50),
                     "cell_updates_per_s": 128 ** 3 * info["steps"] / pct(lat, 50), **info}
    return out


def lagrange128(steps=100, warmup=10):
    import torch
    from paper_2209_01983_amd import sale

    n = 128
    cfg = sale.make_config(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0, mode=sale.SALE_LAGRANGIAN, c_hg=0.1)
    r = sale.SaleRun(cfg, sale.sedov_problem())
    r.step(warmup)
    torch.cuda.synchronize()
    ms = r.step_timed(steps)
    t, nstep, _, flags = r.state()
    if flags:
        raise RuntimeError(f"lagrangian sedov flags {flags}")
    per = sum(ms) / steps
    return {"workload": "sedov 128^3 pure Lagrangian (moving mesh), fp64, hourglass 0.1",
            "steps": steps, "ms_per_step": per, "cell_updates_per_s": n ** 3 * 1e3 / per,
            "kernel_ms": {"begin": ms[0] / steps, "forces+nodes": ms[1] / steps, "energy+geometry": ms[2] / steps},
            "sim_time_end_of_window": t}


def _with_pool_mode(env, fn):
    """Run fn() with pools created under the environment settings `env`
    (the library reads SALE_POOL_PERSISTENT and SALE_POOL_GRAPHS when a pool
    is created)."""
    old = {k: os.environ.get(k) for k in env}
    for k, v in env.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


POOL_MODES = (("persistent", {"SALE_POOL_PERSISTENT": "1"}),
              ("lockstep", {"SALE_POOL_PERSISTENT": "0", "SALE_POOL_GRAPHS": "1"}),
              ("lockstep_launched", {"SALE_POOL_PERSISTENT": "0", "SALE_POOL_GRAPHS": "0"}),
              ("default", {"SALE_POOL_PERSISTENT": None, "SALE_POOL_GRAPHS": None}))


def batched(seq_fp64=True, modes=None, steps=200, runs=256, edge=(16, 64)):
    from paper_2209_01983_amd import sale, workloads
    from paper_2209_01983_amd.inputs import BATCH_SEED, batch_mix

    reqs = batch_mix(runs, seed=BATCH_SEED, edge=edge)
    modes = [m for m, _ in POOL_MODES] if modes is None else modes
    out = {"workload": f"{runs} runs, edges {edge[0]}..{edge[1]} (seed 2209), {runs // 2} sod + {runs - runs // 2} "
                       f"sedov, {steps} steps, one pool advance",
           "cells_total": sum(workloads.cells(r) for r in reqs),
           "modes": {"persistent": "one launch of the persistent kernel per advance (each run served by the "
                                   "blocks of one XCD, work items pulled from per-XCD device queues, per-run "
                                   "phase waits)",
                     "lockstep": "per step: one kernel each for dt, the Lagrange tiles of all runs, the remap "
                                 f"tiles of all runs and the clocks; the first step launched, the other {steps - 1} "
                                 "replays of one captured HIP graph of a step",
                     "lockstep_launched": "the lockstep kernels, every step launched (no graph)",
                     "default": "no mode forced: the library's choice (persistent with at least four runs per "
                                "XCD and balanced XCD loads, lockstep launched otherwise)"}}
    for mode, env in POOL_MODES:
        if mode not in modes:
            continue
        def one(prec):
            r = workloads.run_batched(reqs, steps, prec)
            r["pool"].close()
            return {"cell_updates_per_s": r["cell_updates_per_s"], "makespan_s": r["makespan_s"],
                    "latency_p50_s": pct(r["latency_s"], 50), "latency_p99_s": pct(r["latency_s"], 99)}

        def both():
            # one untimed warm-up advance on a small batch (code objects, clocks)
            workloads.run_batched(reqs[:8], 5, sale.SALE_MIXED32)["pool"].close()
            return {"mixed32": one(sale.SALE_MIXED32), "fp64": one(sale.SALE_FP64)}

        say("batched", mode)
        out[mode] = _with_pool_mode(env, both)
    # the headline figures of the block: the persistent launch
    if "persistent" in out:
        out["mixed32"], out["fp64"] = out["persistent"]["mixed32"], out["persistent"]["fp64"]
    if seq_fp64:
        wall, cps, lat = workloads.run_sequential(reqs, steps, sale.SALE_FP64)
        out["fp64_sequential_plain"] = {"cell_updates_per_s": cps, "wall_s": wall,
                                        "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99)}
    return out


def serving(n_req, budget_gb):
    from paper_2209_01983_amd import sale, workloads
    from paper_2209_01983_amd.inputs import SERVE_SEED, serve_trace

    trace = serve_trace(n_req, seed=SERVE_SEED)
    out = {"workload": f"{n_req} requests, Poisson 50/s (seed 1983), cubic 32..192, 100..500 steps, "
                       f"50/50 sod/sedov, budget {budget_gb:g} GB, fields copied to the host",
           "offered_cell_updates_per_s": sum(workloads.cells(r) * r["steps"] for r in trace)
           / trace[-1]["arrival"]}
    # arrival order with every request admitted as memory allows (throughput
    # first), then shortest job first with at most 24 M cells in flight (a
    # short request waits less and shares the GPU with fewer others)
    for name, prec, kw in (("mixed32", sale.SALE_MIXED32, {}), ("fp64", sale.SALE_FP64, {}),
                           ("mixed32_sjf_24Mcells", sale.SALE_MIXED32, {"order": "sjf", "max_cells": 24_000_000})):
        say("serving", name)
        _, st = workloads.serve(trace, prec, int(budget_gb * 2 ** 30), **kw)
        out[name] = st
    return out


def copy_calibration(nbytes=2 << 30):
    """One plain device-to-device copy kernel of `nbytes` (read nbytes, write
    nbytes): the reference that scales the HBM byte counters."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    say("copy calibration", nbytes, "bytes")


def precision_report(n):
    """Sedov n^3 to t = 1.0 in FP64 and in MIXED32; per-field L1-relative
    (sum |a - b| / sum |b|) and Linf-relative (max |a - b| / max |b|; the
    velocity components against the largest speed component) errors of the
    MIXED32 fields against the FP64 ones, run times and steps."""
    import numpy as np
    import torch
    from paper_2209_01983_amd import sale

    out = {"workload": f"sedov {n}^3 to t=1.0"}
    fields = {}
    for name, prec in (("fp64", sale.SALE_FP64), ("mixed32", sale.SALE_MIXED32)):
        cfg = sale.make_config(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0, precision=prec)
        r = sale.SaleRun(cfg, sale.sedov_problem())
        torch.cuda.synchronize()
        a = time.perf_counter()
        while True:  # in slices, with a progress line after each
            rc = r.run(max_steps=2000)
            t, steps, _, _ = r.state()
            say(f"precision report {name}: t = {t:.4f} after {steps} steps, {time.perf_counter() - a:.1f} s")
            if rc != sale.SALE_OK:
                break
        wall = time.perf_counter() - a
        if rc != sale.SALE_DONE:
            raise RuntimeError(f"{name} run ended with {rc}")
        m, e = r.totals()
        fields[name] = r.fields()
        out[name] = {"steps": steps, "wall_s": wall, "cell_updates_per_s": n ** 3 * steps / wall,
                     "mass": m, "energy": e}
        r.close()
    a, b = fields["mixed32"], fields["fp64"]
    vs = max(np.abs(b[k]).max() for k in ("u", "v", "w"))
    spd = np.sqrt(b["u"] ** 2 + b["v"] ** 2 + b["w"] ** 2)
    # cell by cell: |a - b| / max(|b|, floor), floors the background density
    # and energy of the Sedov set-up and 1e-3 of the largest speed component
    floors = {"rho": 1.0, "e": 1e-6 / (0.4 * 1.0), "u": 1e-3 * vs}
    err = {}
    for k in ("rho", "e", "u", "v", "w"):
        d = np.abs(a[k] - b[k])
        scale = vs if k in ("u", "v", "w") else np.abs(b[k]).max()
        ref = np.maximum(spd, floors["u"]) if k in ("u", "v", "w") else np.maximum(np.abs(b[k]), floors[k])
        r = d / ref
        err[k] = {"l1_rel": float(d.sum() / max(np.abs(b[k]).sum(), 1e-300)),
                  "linf_rel": float(d.max() / max(scale, 1e-300)),
                  "cell_rel_quantiles": {q: float(np.quantile(r, p))
                                         for q, p in (("p50", 0.5), ("p99", 0.99), ("p999", 0.999), ("max", 1.0))}}
    out["mixed32_vs_fp64"] = err
    out["note"] = ("MIXED32 against the FP64 path (which matches the FP64 oracle to 1e-12 per field per step); "
                   "linf_rel against each field's largest value (velocity: the largest speed component); "
                   "cell_rel against max(|fp64|, floor): background rho 1, background e 2.5e-6, "
                   "1e-3 of the largest speed component")
    return out


def host_cpu():
    """Model name and CPU counts of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_in_affinity": affinity}


def cpu_sedov_leg(o, s, n, steps, threads=None):
    """`steps` FP64 oracle steps of the Sedov n^3 workload on `threads`
    OpenMP threads (None: the process default): (cell-updates/s, threads, s)."""
    from oracle import oracle as orc

    if threads:
        orc.set_threads(threads)
    used = orc.max_threads()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, _ = o.step(s)
        assert rc == orc.OK
    dt = time.perf_counter() - t0
    return n ** 3 * steps / dt, used, dt


def cpu_baseline(n, steps_all, steps_one, sod_reps):
    """The FP64 oracle on this host: the Sedov n^3 workload on all threads
    (after one warm-up step) and on one thread, and the whole Sod 64x4x4 run
    to t = 0.2 (full-run latency)."""
    from oracle import oracle as orc

    default_threads = orc.max_threads()
    g = orc.Grid(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0)
    s = orc.sedov(g)
    o = orc.Oracle(g)
    o.step(s)
    say("cpu oracle: all threads")
    cps, threads, secs = cpu_sedov_leg(o, s, n, steps_all)
    say("cpu oracle: one thread")
    cps1, _, secs1 = cpu_sedov_leg(o, s, n, steps_one, threads=1)
    orc.set_threads(default_threads)
    o.close()
    say("cpu oracle: sod latency")
    gs = orc.Grid(64, 4, 4, hi=(1.0, 0.0625, 0.0625), t_end=0.2)
    lat, nsteps = [], 0
    for _ in range(sod_reps + 2):
        a = time.perf_counter()
        os_ = orc.sod(gs)
        osc = orc.Oracle(gs)
        rc, nsteps = osc.run(os_)
        b = time.perf_counter()
        assert rc == orc.DONE
        osc.close()
        lat.append(b - a)
    lat = lat[2:]
    return {"value": cps, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps_all} FP64 oracle steps of the same {n}^3 Sedov workload on {threads} OpenMP "
                      f"threads after 1 warm-up step ({secs:.1f} s)",
            "host": host_cpu(),
            "one_thread": {"value": cps1, "unit": "cell-updates/s", "cores": 1,
                           "sample": f"{steps_one} oracle steps of the {n}^3 Sedov workload ({secs1:.1f} s)"},
            "sod64_latency": {"workload": "sod 64x4x4 to t=0.2, whole oracle run (init + steps)",
                              "cores": threads, "runs": sod_reps, "steps": nsteps,
                              "p50_ms": pct(lat, 50) * 1e3, "p99_ms": pct(lat, 99) * 1e3}}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the SALE step here is a single-GPU path "
              "(multi-GPU halo exchange is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    from paper_2209_01983_amd import sale

    if a.section:
        block = {"latency": lambda: sod_latency(50), "sedov128": lambda: sedov128(3), "noh128": lambda: noh128(3),
                 "lagrange128": lagrange128,
                 "batched": lambda: batched(not a.no_seq, a.pool_modes.split(","), a.batched_steps, a.batch_runs,
                                            tuple(int(x) for x in a.batch_edge.split(","))),
                 "serving": lambda: serving(a.serve_requests, a.serve_budget_gb)}[a.section]
        print(json.dumps({a.section: block()}), flush=True)
        return
    if a.copy_calibration:
        copy_calibration()
    n = a.n
    say("headline fp64", n)
    fixed = tuple(int(x) for x in a.shape.split(",")) if a.shape else None
    ms, t_sim, k64, shape64 = headline(n, a.steps, a.warmup, sale.SALE_FP64, tuned=not a.no_tune, fixed=fixed)
    say("headline mixed32", n)
    ms32, _, k32, shape32 = headline(n, a.steps, a.warmup, sale.SALE_MIXED32, tuned=not a.no_tune, fixed=fixed)
    cells = n ** 3
    value = cells * 1e3 / ms
    abytes = algorithmic_bytes(n)
    step_kernel_ms = sum(k64)
    achieved = abytes / (step_kernel_ms * 1e-3) / 1e9
    comp = compulsory_bytes(n)
    traffic, traffic_note = measured_traffic(n, shape64)
    kernels = []
    for name, kms in (("k_begin", k64[0]), ("k_lagrange", k64[1]), ("k_remap", k64[2])):
        b = comp.get(name)
        kernels.append({"name": name, "avg_ms": kms,
                        "compulsory_bytes": b, "compulsory_GBps": (b / (kms * 1e-3) / 1e9) if b else None})
    dominant = max(kernels, key=lambda k: k["avg_ms"])
    out = {
        "metric": "cell-updates/s (Lagrange+remap) 320^3 FP64 vs FP32; p50/p99 per-run latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Sedov blast initial state generated on the device)",
        "config": {"workload": f"sedov {n}^3 octant of [0,1.2]^3, FP64 Lagrange + donor-cell remap, CFL 0.5",
                   "cells": cells, "precision": "fp64", "sim_time_end_of_window": t_sim,
                   "launch_shape": shape64},
        "mixed32": {"value": cells * 1e3 / ms32, "unit": "cell-updates/s", "ms_per_step": ms32,
                    "kernel_ms": k32, "launch_shape": shape32,
                    "precision": "FP32 bulk, FP64 geometry/volumes/dt/totals"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic / (step_kernel_ms * 1e-3) / 1e9) if traffic else None,
                     "traffic_bytes_per_step": traffic, "traffic_source": traffic_note,
                     "unit_of_work": "one step (k_begin + k_lagrange + k_remap), HIP events per kernel",
                     "algorithmic_bytes_per_cell": abytes / cells,
                     "step_kernel_ms": step_kernel_ms, "dominant_kernel": dominant["name"],
                     "kernels": kernels},
    }
    say("headline fp64, second-order remap", n)
    ms2, _, k2, _ = headline(n, a.steps, a.warmup, sale.SALE_FP64, tuned=False,
                             fixed=(shape64["rows_a"], shape64["rows_b"], shape64["target"]), order=2)
    out["remap_order2"] = {"value": cells * 1e3 / ms2, "unit": "cell-updates/s", "ms_per_step": ms2,
                           "kernel_ms": {"k_begin": k2[0], "k_lagrange": k2[1], "remap (3 passes)": k2[2]},
                           "precision": "fp64", "note": "limited linear donor values; three z-marching tile passes"}
    if not a.quick:
        say("sod latency")
        out["latency"] = sod_latency(50)
        say("sedov 128")
        out["sedov128"] = sedov128(3)
        say("noh 128")
        out["noh128"] = noh128(3)
        say("lagrange 128")
        out["lagrange128"] = lagrange128()
        say("batched")
        out["batched"] = batched()
        out["serving"] = serving(a.serve_requests, a.serve_budget_gb)
    prec_n = a.precision_report if a.precision_report is not None else (0 if a.quick else 128)
    if prec_n:
        say("precision report", prec_n)
        out["precision"] = precision_report(prec_n)
    if not a.no_cpu:
        say("cpu oracle")
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_steps, a.cpu_steps_one, 50)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
