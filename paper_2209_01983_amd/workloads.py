"""Multi-run workloads on the library's pool: the batched launch and the
continuous-batching server, and the problem set-up both use.

Problem set-up of a multi-run request (cubic cells of edge h):
  Sod:   h = 1/nx, box [0,1] x [0,ny h] x [0,nz h], split at x = 0.5, left
         rho = 1, p = 1, right rho = 1/r_rho, p = 1/r_p, u = 0.
  Sedov: h = 1.2/max(nx,ny,nz), box [0,nx h] x [0,ny h] x [0,nz h], rho = 1,
         p = 1e-6, the drawn energy deposited in the corner cell (0,0,0).
The runs stop after their step count (the end time is set out of reach).

Every step of every run executes in the library's kernels; this module only
admits runs, calls the pool and keeps the clock.
"""
import collections
import time

from . import sale

T_FAR = 1e30  # end time out of reach: multi-run requests stop on their step count


def request_problem(req, precision):
    """(config, problem) of one batched / served request (see module doc)."""
    nx, ny, nz = req["n"]
    if req["kind"] == "sod":
        h = 1.0 / nx
        cfg = sale.make_config(nx, ny, nz, hi=(1.0, ny * h, nz * h), t_end=T_FAR, precision=precision)
        prob = sale.sod_problem(0.5, 1.0, 1.0, 1.0 / req["rho_ratio"], 1.0 / req["p_ratio"])
    else:
        h = 1.2 / max(nx, ny, nz)
        cfg = sale.make_config(nx, ny, nz, hi=(nx * h, ny * h, nz * h), t_end=T_FAR, precision=precision)
        prob = sale.sedov_problem(1.0, 1e-6, req["edep"])
    return cfg, prob


def cells(req):
    nx, ny, nz = req["n"]
    return nx * ny * nz


def arena_bytes_for(reqs, precision, slack=1 << 20):
    return sum(sale.sale_workspace_bytes(request_problem(r, precision)[0]) for r in reqs) + slack


def run_batched(reqs, steps, precision, pool=None):
    """All requests admitted into one pool and advanced by ONE pool advance
    of `steps` steps (lockstep launches over all runs, or the persistent
    kernel). Returns a dict: makespan (s, HIP events around the advance), aggregate cell-updates/s, per-run latency (s, from the
    launch's first wave to the run's last completed step, device clock), and
    the pool with its slots (for result checks)."""
    import torch

    if pool is None:
        pool = sale.Pool(arena_bytes_for(reqs, precision) + (64 << 20), max_runs=len(reqs), precision=precision)
    slots = []
    for r in reqs:
        cfg, prob = request_problem(r, precision)
        s = pool.admit(cfg, prob, steps)
        if s is None:
            raise RuntimeError("batched pool too small")
        slots.append(s)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pool.advance(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    makespan = e0.elapsed_time(e1) * 1e-3
    done = pool.poll()
    if sorted(done) != sorted(slots):
        raise RuntimeError(f"batched launch left runs unfinished ({len(done)} of {len(slots)})")
    clocks = [pool.clock(s) for s in slots]
    t0 = min(c[0] for c in clocks)
    lat = [c[1] - t0 for c in clocks]
    for s in slots:
        t, n, _, flags = pool.state(s)
        if n != steps or flags:
            raise RuntimeError(f"slot {s}: {n} steps, flags {flags}")
    total = sum(cells(r) for r in reqs) * steps
    return {"makespan_s": makespan, "cell_updates_per_s": total / makespan, "latency_s": lat,
            "pool": pool, "slots": slots}


def run_sequential(reqs, steps, precision):
    """The same requests one after another on the single-run path (one
    context each, `steps` steps, synchronised at the end of each run).
    Returns (wall seconds, aggregate cell-updates/s, per-run latency list)."""
    import torch

    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        a = time.perf_counter()
        cfg, prob = request_problem(r, precision)
        run = sale.SaleRun(cfg, prob)
        run.step(steps)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        run.close()
    wall = time.perf_counter() - t0
    return wall, sum(cells(r) for r in reqs) * steps / wall, lat


Served = collections.namedtuple("Served", "index arrival admitted finished slot fields")


def serve(trace, precision, budget_bytes, max_runs=512, slice_steps=25, keep=None, fetch=True,
          clock=time.perf_counter, sleep=time.sleep, max_cells=None, order="fifo"):
    """Continuous-batching server over a request trace (dicts with arrival
    time in s, kind, n, steps and the problem parameters).

    Requests enter a queue at their arrival time; its head is admitted into
    the pool whenever a slot and an arena range of the HBM budget are free
    (admission refuses otherwise, and the head waits). The queue is in
    arrival order (`order="fifo"`) or, with `order="sjf"`, in order of the
    work a request asks for (cells x steps, shortest first; ties by arrival),
    which cuts the median latency when requests wait. With
    `max_cells`, while the admitted runs hold fewer cells than that (a cap on
    how many runs share the GPU at once: fewer runs in flight finish sooner
    each, as long as they still fill the chip). Admitted runs
    advance together, `slice_steps` steps per pool advance; between
    launches finished runs are polled, their fields copied to the host (the
    result a client receives), their memory released, and newly arrived
    requests admitted. Latency = arrival -> fields on the host.

    `keep` (set of request indices) selects whose fields are returned.
    Returns (list of Served, stats dict)."""
    import numpy as np

    if order not in ("fifo", "sjf"):
        raise ValueError(f"order must be 'fifo' or 'sjf', not {order!r}")
    pool = sale.Pool(budget_bytes, max_runs=max_runs, precision=precision)
    pending = collections.deque(enumerate(trace))
    queue = collections.deque()
    active = {}          # slot -> (index, arrival, admitted)
    active_cells = 0
    out = []
    busy_cells = 0       # cell-updates executed
    t_start = clock()
    launches = 0
    while pending or queue or active:
        now = clock() - t_start
        arrived = False
        while pending and pending[0][1]["arrival"] <= now:
            queue.append(pending.popleft())
            arrived = True
        if arrived and order == "sjf":
            queue = collections.deque(sorted(queue, key=lambda q: (cells(q[1]) * q[1]["steps"], q[0])))
        while queue:
            i, req = queue[0]
            if max_cells is not None and active and active_cells + cells(req) > max_cells:
                break
            cfg, prob = request_problem(req, precision)
            slot = pool.admit(cfg, prob, req["steps"])
            if slot is None:
                if not active:
                    raise RuntimeError(f"request {i} does not fit the budget even alone")
                break
            queue.popleft()
            active[slot] = (i, req["arrival"], clock() - t_start)
            active_cells += cells(req)
        if not active:
            if pending:
                wait = pending[0][1]["arrival"] - (clock() - t_start)
                if wait > 0:
                    sleep(wait)
            continue
        pool.advance(slice_steps)
        launches += 1
        for slot in pool.poll():
            i, arr, adm = active.pop(slot)
            req = trace[i]
            active_cells -= cells(req)
            fields = pool.fields(slot) if fetch or (keep and i in keep) else None
            t, n, _, flags = pool.state(slot)
            fin = clock() - t_start
            if n != req["steps"] or flags:
                raise RuntimeError(f"request {i}: {n} of {req['steps']} steps, flags {flags}")
            busy_cells += cells(req) * req["steps"]
            if keep is not None and i not in keep:
                fields = None
            out.append(Served(i, arr, adm, fin, slot, fields))
            pool.release(slot)
    wall = clock() - t_start
    pool.close()
    lat = np.array([s.finished - s.arrival for s in out])
    qd = np.array([s.admitted - s.arrival for s in out])
    stats = {"requests": len(out), "wall_s": wall, "cell_updates_per_s": busy_cells / wall,
             "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
             "queue_p50_s": float(np.percentile(qd, 50)), "queue_p99_s": float(np.percentile(qd, 99)),
             "launches": launches, "slice_steps": slice_steps, "budget_bytes": budget_bytes,
             "max_cells": max_cells, "order": order}
    return sorted(out, key=lambda s: s.index), stats
