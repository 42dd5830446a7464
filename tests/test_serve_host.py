"""Host logic of the continuous-batching server (no GPU): FIFO and
shortest-job-first admission under a budget, slicing, completion, release
and latency accounting, with the pool replaced by a stand-in that only
counts steps."""
import pytest

from paper_2209_01983_amd import sale, workloads


class CountingPool:
    """Stand-in for sale.Pool: a run needs `cells` bytes of the budget and
    finishes after its step count; nothing is computed."""
    log = []

    def __init__(self, budget, max_runs, precision):
        self.budget, self.max_runs, self.used = budget, max_runs, 0
        self.runs = {}

    def admit(self, cfg, prob, n_steps):
        need = cfg.nx * cfg.ny * cfg.nz
        if self.used + need > self.budget or len(self.runs) >= self.max_runs:
            return None
        slot = min(set(range(self.max_runs)) - set(self.runs))
        self.runs[slot] = [need, n_steps, 0]
        self.used += need
        CountingPool.log.append(("admit", slot, cfg.nx))
        return slot

    def advance(self, k):
        for r in self.runs.values():
            r[2] = min(r[1], r[2] + k)

    def poll(self):
        out = [s for s, r in self.runs.items() if r[2] >= r[1] and len(r) == 3]
        for s in out:
            self.runs[s].append("reported")
        return out

    def fields(self, slot):
        return {"steps": self.runs[slot][2]}

    def state(self, slot):
        r = self.runs[slot]
        return 0.0, r[2], 0.0, 0

    def release(self, slot):
        self.used -= self.runs.pop(slot)[0]

    def close(self):
        pass


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t

    def sleep(self, dt):
        self.t += dt


def trace_of(sizes_steps, gap=0.01):
    return [{"arrival": gap * i, "kind": "sedov", "n": (n, n, n), "steps": s, "edep": 0.5}
            for i, (n, s) in enumerate(sizes_steps)]


def test_fifo_admission_under_budget_and_latency_accounting(monkeypatch):
    monkeypatch.setattr(sale, "Pool", CountingPool)
    CountingPool.log = []
    tr = trace_of([(4, 10), (4, 30), (4, 5), (2, 5), (3, 7)])
    clk = FakeClock()
    # budget: two 4^3 runs at once
    served, st = workloads.serve(tr, sale.SALE_FP64, 2 * 64 + 10, max_runs=4, slice_steps=5, clock=clk,
                                 sleep=clk.sleep)
    assert [s.index for s in served] == [0, 1, 2, 3, 4]
    assert all(s.fields["steps"] == tr[s.index]["steps"] for s in served)
    admitted = [e[2] for e in CountingPool.log]
    assert admitted == [4, 4, 4, 2, 3]          # FIFO: request 3 does not overtake request 2
    for s in served:
        assert s.arrival <= s.admitted <= s.finished
    assert served[2].admitted > served[2].arrival  # waited for memory
    assert st["requests"] == 5 and st["latency_p99_s"] >= st["latency_p50_s"] > 0
    assert st["cell_updates_per_s"] > 0


def test_shortest_job_first_admits_the_smallest_waiting_request(monkeypatch):
    monkeypatch.setattr(sale, "Pool", CountingPool)
    CountingPool.log = []
    # all arrive at once; the budget holds one 4^3 run or several small ones
    tr = trace_of([(4, 20), (4, 30), (2, 50), (3, 5), (2, 10)], gap=0.0)
    clk = FakeClock()
    served, st = workloads.serve(tr, sale.SALE_FP64, 64 + 10, max_runs=4, slice_steps=5, clock=clk,
                                 sleep=clk.sleep, order="sjf")
    admitted = [(e[2]) for e in CountingPool.log]
    # work = cells x steps: 2^3*10=80 < 3^3*5=135 < 2^3*50=400 < 4^3*20 < 4^3*30
    assert admitted == [2, 3, 2, 4, 4]
    assert all(s.fields["steps"] == tr[s.index]["steps"] for s in served)
    assert st["order"] == "sjf"
    with pytest.raises(ValueError):
        workloads.serve(tr, sale.SALE_FP64, 1000, clock=clk, sleep=clk.sleep, order="lifo")


def test_idle_server_sleeps_until_the_next_arrival(monkeypatch):
    monkeypatch.setattr(sale, "Pool", CountingPool)
    tr = trace_of([(2, 3), (2, 3)], gap=5.0)
    clk = FakeClock()
    served, st = workloads.serve(tr, sale.SALE_FP64, 1000, clock=clk, sleep=clk.sleep)
    assert served[1].admitted >= 5.0 and st["launches"] == 2


def test_request_larger_than_the_budget_is_an_error(monkeypatch):
    monkeypatch.setattr(sale, "Pool", CountingPool)
    tr = trace_of([(8, 3)])
    clk = FakeClock()
    with pytest.raises(RuntimeError, match="does not fit"):
        workloads.serve(tr, sale.SALE_FP64, 100, clock=clk, sleep=clk.sleep)


def test_request_geometry_follows_the_stated_setup():
    cfg, prob = workloads.request_problem({"kind": "sod", "n": (40, 8, 4), "rho_ratio": 8.0, "p_ratio": 10.0},
                                          sale.SALE_MIXED32)
    assert tuple(cfg.hi) == pytest.approx((1.0, 0.2, 0.1)) and cfg.precision == sale.SALE_MIXED32
    assert list(prob.sod) == pytest.approx([0.5, 1.0, 1.0, 0.125, 0.1])
    cfg, prob = workloads.request_problem({"kind": "sedov", "n": (20, 40, 30), "edep": 0.3}, sale.SALE_FP64)
    assert tuple(cfg.hi) == pytest.approx((0.6, 1.2, 0.9))
    assert list(prob.sedov) == pytest.approx([1.0, 1e-6, 0.3])


def test_tuner_choice_and_cache_round_trip(tmp_path, monkeypatch):
    from paper_2209_01983_amd import tune
    times = {(8, 1024): (3.0, 2.0), (16, 1024): (1.0, 2.5), (32, 1024): (1.5, 1.8),
             (8, 2048): (2.0, 1.0), (16, 2048): (1.2, 1.1), (32, 2048): (1.4, 1.3)}
    best = tune.choose(times)
    # target 1024: 1.0 + 1.8 = 2.8; target 2048: 1.2 + 1.0 = 2.2
    assert (best["rows_a"], best["rows_b"], best["target"]) == (16, 8, 2048)
    assert best["ms"] == pytest.approx(2.2)
    path = str(tmp_path / "c.json")
    cfg = sale.make_config(20, 30, 40, precision=sale.SALE_MIXED32)
    monkeypatch.setattr(tune, "arch", lambda: "gfx950")
    cache = {tune.key("gfx950", "lagrange", cfg): {"rows": 32, "target": 6144, "ms": 1.0},
             tune.key("gfx950", "remap", cfg): {"rows": 8, "target": 6144, "ms": 1.0}}
    tune.save_cache(cache, path)
    assert tune.lookup(cfg, path) == {"rows_a": 32, "rows_b": 8, "target": 6144}
    assert tune.key("gfx950", "remap", cfg) == f"gfx950|remap|20x30x40|mixed32|order1|eulerian|{tune.source_digest()}"
    assert tune.lookup(sale.make_config(20, 30, 41), path) is None
    # remap order and mode are part of the key: an order-2 or Lagrangian run
    # of the same mesh does not pick up this entry
    assert tune.lookup(sale.make_config(20, 30, 40, precision=sale.SALE_MIXED32, remap_order=2), path) is None
    assert tune.lookup(sale.make_config(20, 30, 40, precision=sale.SALE_MIXED32, mode=sale.SALE_LAGRANGIAN),
                       path) is None
    # and an entry dies with the kernel sources it was timed on
    monkeypatch.setattr(tune, "_DIGEST", "0000000000000000")
    assert tune.lookup(cfg, path) is None
