"""GPU tests of the persistent pool advance's XCD queues.

The persistent kernel serves every run from the blocks of one XCD (the runs
are spread over the XCDs the device reports, balanced by cells). Bars: runs
packed onto one XCD give bitwise the results of the same runs spread over all
of them; a run assigned to an XCD that receives no block of the launch is
flagged (SALE_FLAG_NUMERIC) by the last block to leave, and the advance ends
normally (nothing waits for that XCD). SALE_POOL_XCC_MASK, read at pool
creation, sets the XCDs the host assigns runs to.
"""
import numpy as np
import pytest

from paper_2209_01983_amd import sale
from paper_2209_01983_amd.inputs import random_state

from parity import FIELDS, say  # noqa: E402

pytestmark = pytest.mark.gpu

ARENA = 256 << 20
SHAPES = ((33, 26, 40), (7, 7, 7), (64, 5, 3), (20, 48, 2), (17, 17, 17), (40, 9, 12), (3, 30, 30),
          (50, 50, 4), (1, 1, 1), (29, 31, 37))


def run_pool(monkeypatch, mask, steps=12, precision=sale.SALE_FP64):
    monkeypatch.setenv("SALE_POOL_PERSISTENT", "1")
    if mask is None:
        monkeypatch.delenv("SALE_POOL_XCC_MASK", raising=False)
    else:
        monkeypatch.setenv("SALE_POOL_XCC_MASK", hex(mask))
    pool = sale.Pool(ARENA, max_runs=len(SHAPES), precision=precision)
    keep, slots = [], []
    for i, n in enumerate(SHAPES):
        st = random_state(*n, seed=40 + i, smooth=True)
        cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0, precision=precision)
        p, k = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"])
        keep.append(k)
        slots.append(pool.admit(cfg, p, steps))
    pool.advance(5)
    pool.advance(steps)
    done = pool.poll()
    out = {s: (pool.state(s), pool.fields(s)) for s in slots}
    pool.close()
    return out, done


@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_runs_on_one_xcd_match_runs_spread_over_all(monkeypatch, precision):
    say("pool xcd: one XCD vs all, precision", precision)
    ref, done_ref = run_pool(monkeypatch, None, precision=precision)
    got, done = run_pool(monkeypatch, 0x1, precision=precision)
    assert sorted(done) == sorted(done_ref) == sorted(ref)
    for s in ref:
        (st_r, f_r), (st_g, f_g) = ref[s], got[s]
        assert st_r[3] == 0 and st_g == st_r, (s, st_g, st_r)
        assert st_r[1] == 12
        for k in FIELDS:
            assert np.array_equal(f_g[k], f_r[k]), (s, k)


def test_runs_of_an_xcd_without_blocks_are_flagged(monkeypatch):
    # XCD id 15: none on this device (MI355X reports ids 0..7)
    say("pool xcd: runs on an XCD that receives no block")
    got, done = run_pool(monkeypatch, 1 << 15)
    assert sorted(done) == sorted(got)
    for s, (st, _) in got.items():
        assert st[3] & sale.SALE_FLAG_NUMERIC, (s, st)


def test_default_mode_on_many_runs_matches_lockstep(monkeypatch):
    """40 runs of one size: five per XCD, so the advance takes the persistent
    kernel when no mode is forced; results bitwise those of forced lockstep."""
    say("pool xcd: default mode on 40 equal runs vs lockstep")
    n = (18, 11, 9)

    def go(mode):
        if mode is None:
            monkeypatch.delenv("SALE_POOL_PERSISTENT", raising=False)
        else:
            monkeypatch.setenv("SALE_POOL_PERSISTENT", mode)
        monkeypatch.delenv("SALE_POOL_XCC_MASK", raising=False)
        pool = sale.Pool(ARENA, max_runs=40)
        keep, slots = [], []
        for i in range(40):
            st = random_state(*n, seed=100 + i, smooth=True)
            cfg = sale.make_config(*n, hi=(1.0, 0.6, 0.5), t_end=100.0)
            p, k = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"])
            keep.append(k)
            slots.append(pool.admit(cfg, p, 9))
        pool.advance(4)
        pool.advance(9)
        assert sorted(pool.poll()) == sorted(slots)
        out = {s: (pool.state(s), pool.fields(s)) for s in slots}
        pool.close()
        return out

    ref, got = go("0"), go(None)
    for s in ref:
        assert ref[s][0][3] == 0 and got[s][0] == ref[s][0], s
        for k in FIELDS:
            assert np.array_equal(got[s][1][k], ref[s][1][k]), (s, k)


def test_capped_waits_abort_the_advance_and_flag_their_runs(monkeypatch):
    """A wait cap of 0 ticks (set from the host) makes the first wait that is
    not satisfied at once time out: the advance aborts, later waits give up,
    the runs whose items could not wait are flagged SALE_FLAG_NUMERIC, and
    the launch ends normally. A run left unflagged completed every step of
    the advance and matches the same run in a pool without the cap bitwise."""
    say("pool xcd: capped waits abort the advance")
    ref, _ = run_pool(monkeypatch, None)
    monkeypatch.setenv("SALE_POOL_WAIT_TICKS", "0")
    got, done = run_pool(monkeypatch, None)
    monkeypatch.delenv("SALE_POOL_WAIT_TICKS")
    assert sorted(done) == sorted(got)
    flagged = [s for s, (st, _) in got.items() if st[3] & sale.SALE_FLAG_NUMERIC]
    assert flagged, "no wait hit a cap of 0 ticks"
    for s, (st, f) in got.items():
        if s in flagged:
            continue
        assert st == ref[s][0], (s, st, ref[s][0])
        for k in FIELDS:
            assert np.array_equal(f[k], ref[s][1][k]), (s, k)


@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_batched_256_runs_persistent_bitwise_equals_lockstep(monkeypatch, precision):
    """The benchmark's batch (256 runs, edges 16..64) advanced 40 steps by one
    persistent launch gives every run bitwise the fields and clocks-free state
    of the lockstep kernels: thousands of tile hand-offs per step through the
    XCDs' L2s."""
    import torch
    from paper_2209_01983_amd import workloads
    from paper_2209_01983_amd.inputs import BATCH_SEED, batch_mix

    say("pool xcd: 256-run batch, persistent vs lockstep, precision", precision)
    reqs = batch_mix(256, seed=BATCH_SEED)
    monkeypatch.delenv("SALE_POOL_XCC_MASK", raising=False)
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("SALE_POOL_PERSISTENT", mode)
        r = workloads.run_batched(reqs, 40, precision)
        pool = r["pool"]
        out[mode] = [(pool.state(s), pool.fields(s, on_device=True)) for s in r["slots"]]
        pool.close()
    for (st_p, f_p), (st_l, f_l) in zip(out["1"], out["0"]):
        assert st_p == st_l and st_p[1] == 40 and st_p[3] == 0, (st_p, st_l)
        for k in FIELDS:
            assert torch.equal(f_p[k], f_l[k]), k
