"""GPU test of the pool's graph-replayed lockstep rounds.

In the lockstep mode an advance's first round is launched and every later
round is a replay of one captured graph of a round, kept while the round's
shape (active runs, block counts) stays the same and captured again when it
changes. The bar: the results, clocks and step counts of every run are
bitwise those of the same sequence of advances with every round launched
(SALE_POOL_GRAPHS=0), over advances that reuse the graph, advances after an
admission or a release (a new shape: a new capture), runs that finish inside
an advance (their tiles are skipped in the replays) and one-step advances
(no graph).
"""
import numpy as np
import pytest

from paper_2209_01983_amd import sale
from paper_2209_01983_amd.inputs import random_state

from parity import FIELDS, say  # noqa: E402

pytestmark = pytest.mark.gpu

ARENA = 256 << 20


def scripted(monkeypatch, graphs, precision):
    """One fixed sequence of admissions, advances and releases; the final
    fields and (t, steps, dt, flags) of every slot."""
    monkeypatch.setenv("SALE_POOL_PERSISTENT", "0")
    monkeypatch.setenv("SALE_POOL_GRAPHS", "1" if graphs else "0")
    pool = sale.Pool(ARENA, max_runs=8, precision=precision)
    keep = []

    def admit(n, seed, steps):
        st = random_state(*n, seed=seed, smooth=True)
        cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0, precision=precision)
        p, k = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"])
        keep.append(k)
        return pool.admit(cfg, p, steps)

    slots = [admit((33, 26, 40), 1, 30), admit((7, 7, 7), 2, 5), admit((64, 5, 3), 3, 40)]
    pool.advance(4)     # captured, replayed 3 times
    pool.advance(4)     # same shape: the same graph
    pool.advance(1)     # one round: no replay
    slots.append(admit((20, 48, 2), 4, 25))
    pool.advance(6)     # a new shape: captured again; the 7^3 run finishes inside
    pool.release(slots[1])
    pool.poll()
    pool.advance(64)    # every run finishes inside this advance
    done = pool.poll()
    out = {}
    for s in slots[:1] + slots[2:]:
        out[s] = (pool.state(s), pool.fields(s))
    pool.close()
    return out, done


@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_graph_replayed_rounds_are_bitwise_the_launched_rounds(monkeypatch, precision):
    say("pool graphs vs launched rounds, precision", precision)
    ref, done_ref = scripted(monkeypatch, False, precision)
    got, done = scripted(monkeypatch, True, precision)
    assert sorted(done) == sorted(done_ref)
    assert got.keys() == ref.keys()
    for s in ref:
        (st_r, f_r), (st_g, f_g) = ref[s], got[s]
        assert st_g == st_r, (s, st_g, st_r)
        assert st_r[3] == 0
        for k in FIELDS:
            assert np.array_equal(f_g[k], f_r[k]), (s, k)
    # the runs reached their step targets
    assert sorted(v[0][1] for v in ref.values()) == [25, 30, 40]


def test_pool_destroyed_with_replays_queued(monkeypatch):
    """Destroying a pool right after an advance, its round graph's replays
    still queued on the stream, waits for them before the graph goes; pools
    created afterwards (their arenas may reuse the freed memory) run to
    bitwise equal results."""
    say("pool destroy with queued replays")
    monkeypatch.setenv("SALE_POOL_PERSISTENT", "0")
    monkeypatch.setenv("SALE_POOL_GRAPHS", "1")
    n = (40, 24, 30)
    cfg = sale.make_config(*n, hi=(1.0, 0.6, 0.75), t_end=100.0)

    def run(close_early):
        pool = sale.Pool(ARENA, max_runs=4)
        st = random_state(*n, seed=77, smooth=True)
        p, keep = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"])
        s = pool.admit(cfg, p, 40)
        pool.advance(40)
        if close_early:
            pool.close()  # the 39 replays may still be in flight
            return None
        pool.poll()
        out = pool.fields(s)
        pool.close()
        return out

    run(True)
    a = run(False)
    b = run(False)
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
