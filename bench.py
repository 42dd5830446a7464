#!/usr/bin/env python3
"""Benchmark: cell-updates/s of the SALE Lagrange + remap step on one MI355X.

Workload: the Sedov blast on a 320^3 octant mesh of [0,1.2]^3 (rho = 1,
p = 1e-6, E = 0.125 deposited in the corner cell, gamma 1.4, CFL 0.5),
FP64, synthetic initial state generated on the device. W warm-up steps, then
K timed steps between two stream synchronisations; value = cells x K / time.

Prints one JSON line. `roofline` covers the step's HBM roofline (the step is
a bandwidth-bound stencil; no MFMA): algorithmic bytes = read and write of
the state once per step (rho, e per cell; u, v, w per node, FP64). The CPU
baseline is the FP64 oracle timed on this host's cores on a few steps of the
same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=320, help="cells per axis")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=3)
    return ap.parse_args()


def algorithmic_bytes(n):
    ncell = n ** 3
    nnode = (n + 1) ** 3
    return 2 * (2 * ncell + 3 * nnode) * 8  # read + write rho, e, u, v, w (FP64)


def gpu_bench(n, steps, warmup, precision=0):
    import torch

    from paper_2209_01983_amd import sale

    cfg = sale.make_config(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0, precision=precision)
    run = sale.SaleRun(cfg, sale.sedov_problem())
    run.step(warmup)
    torch.cuda.synchronize()
    t0, s0, _, _ = run.state()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    run.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    t1, s1, _, flags = run.state()
    if s1 - s0 != steps or flags != 0:
        raise RuntimeError(f"timed window did not run {steps} full steps ({s1 - s0}, flags {flags})")
    return ms / steps, wall, t1


def cpu_bench(n, steps):
    """The FP64 oracle on this host (all cores OpenMP), one warm-up step then
    `steps` timed steps of the same Sedov workload."""
    from oracle import oracle as orc

    g = orc.Grid(n, n, n, hi=(1.2, 1.2, 1.2), t_end=1.0)
    s = orc.sedov(g)
    o = orc.Oracle(g)
    o.step(s)
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, _ = o.step(s)
        assert rc == orc.OK
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return n ** 3 * steps / dt, threads, dt


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the SALE step here is a single-GPU path "
              "(multi-GPU halo exchange is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    n = a.n
    ms, wall, t_sim = gpu_bench(n, a.steps, a.warmup, precision=0)
    ms32, _, _ = gpu_bench(n, a.steps, a.warmup, precision=1)
    cells = n ** 3
    value = cells * 1e3 / ms
    abytes = algorithmic_bytes(n)
    achieved = abytes / (ms * 1e-3) / 1e9
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
        "config": {"workload": f"sedov {n}^3 octant, FP64 Lagrange + donor-cell remap", "cells": cells,
                   "precision": "fp64", "sim_time_end_of_window": t_sim},
        "mixed32": {"value": cells * 1e3 / ms32, "unit": "cell-updates/s", "ms_per_step": ms32,
                    "precision": "FP32 bulk, FP64 geometry/dt/totals"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole step (all step kernels), algorithmic bytes "
                               f"{abytes / cells:.2f} B/cell"},
    }
    if not a.no_cpu:
        cps, threads, secs = cpu_bench(n, a.cpu_steps)
        out["cpu_baseline"] = {"value": cps, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
                               "sample": f"{a.cpu_steps} FP64 oracle steps of the same {n}^3 Sedov "
                                         f"workload after 1 warm-up step ({secs:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
