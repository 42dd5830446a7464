"""GPU tests of the pool: many independent runs advanced together, through
the C ABI, in both advance modes (lockstep launches over all runs, and the
persistent multi-run kernel serving each run from one XCD) and with the mode
chosen per advance.

Bars: every pool run matches the FP64 oracle run of the same problem and step
count to 1e-12 per field (the single-run bar); a run's results are bitwise
the same alone in a pool, among other runs of uneven sizes, and on the
single-run path (the arithmetic per cell does not depend on tiling or on
pool-mates); slots and arena ranges are reused after release; admission
refuses with SALE_EBUSY when no slot or no arena range is free (SALE_ENOMEM
for a run that could never fit); an error flag
of one run stops that run only.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2209_01983_amd import sale
from paper_2209_01983_amd.inputs import random_state

from parity import FIELDS, assert_parity, grid_of, oracle_state, say  # noqa: E402

pytestmark = pytest.mark.gpu

ARENA = 256 << 20


@pytest.fixture(autouse=True, params=["lockstep", "persistent", "auto"])
def advance_mode(request, monkeypatch):
    """Every pool test runs with both advance modes forced and with the mode
    chosen per advance (read at pool creation)."""
    if request.param == "auto":
        monkeypatch.delenv("SALE_POOL_PERSISTENT", raising=False)
    else:
        monkeypatch.setenv("SALE_POOL_PERSISTENT", "1" if request.param == "persistent" else "0")
    monkeypatch.delenv("SALE_POOL_XCC_MASK", raising=False)
    return request.param


def user_prob(st):
    p, keep = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"])
    return p, keep


def mix_cases():
    """(cfg, problem-maker, host initial state or None, n_steps): uneven sizes,
    ragged tiles, all three problem kinds."""
    out = []
    for n, seed, steps in (((37, 29, 23), 1, 5), ((1, 1, 1), 3, 2), ((65, 3, 2), 2, 7), ((5, 1, 9), 5, 4),
                           ((30, 31, 17), 7, 9)):
        cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0)
        out.append((cfg, "user", random_state(*n, seed=seed), steps))
    out.append((sale.make_config(40, 4, 4, hi=(1.0, 0.1, 0.1), t_end=0.2), "sod", None, 11))
    out.append((sale.make_config(19, 23, 21, hi=(1.2 * 19 / 23, 1.2, 1.2 * 21 / 23), t_end=1.0), "sedov",
                None, 6))
    return out


def problem_of(kind, st):
    if kind == "sod":
        return sale.sod_problem(), None
    if kind == "sedov":
        return sale.sedov_problem(), None
    return user_prob(st)


def oracle_run(cfg, kind, st, n_steps):
    g = grid_of(cfg)
    s = orc.sod(g) if kind == "sod" else orc.sedov(g) if kind == "sedov" else oracle_state(st)
    o = orc.Oracle(g)
    for _ in range(n_steps):
        rc, _ = o.step(s)
        if rc == orc.DONE:
            break
        assert rc == orc.OK
    return s


def drain(pool, chunk, expect, max_advances=1000):
    """Advance by `chunk` steps at a time until `expect` runs were reported."""
    done = []
    for _ in range(max_advances):
        pool.advance(chunk)
        done += pool.poll()
        if len(done) >= expect:
            return done
    raise AssertionError("pool runs did not finish")


@pytest.mark.parametrize("chunk", [1, 4, 64])
def test_pool_runs_match_oracle(chunk):
    say("pool vs oracle, chunk", chunk)
    pool = sale.Pool(ARENA, max_runs=16)
    cases = mix_cases()
    slots = []
    for cfg, kind, st, steps in cases:
        p, keep = problem_of(kind, st)
        slots.append(pool.admit(cfg, p, steps))
        del keep
    assert None not in slots and len(set(slots)) == len(slots)
    done = drain(pool, chunk, len(slots))
    assert sorted(done) == sorted(slots)
    for slot, (cfg, kind, st, steps) in zip(slots, cases):
        s = oracle_run(cfg, kind, st, steps)
        t, nstep, _, flags = pool.state(slot)
        assert flags == 0 and nstep == s.step, (cfg.nx, cfg.ny, cfg.nz, nstep, s.step)
        assert t == pytest.approx(s.t, rel=1e-14)
        assert_parity(pool.fields(slot), s, what=f"slot {slot} {kind} {(cfg.nx, cfg.ny, cfg.nz)}")


@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_pool_is_bitwise_the_single_run_path_alone_or_in_a_mix(precision):
    say("pool alone / mix / single, precision", precision)
    n = (33, 26, 40)
    st = random_state(*n, seed=11, smooth=True)
    cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0, precision=precision)
    steps = 9
    # single-run path
    p, keep = user_prob(st)
    r = sale.SaleRun(cfg, p, keepalive=keep)
    r.step(steps)
    ref = r.fields()
    ref_state = r.state()
    # alone in a pool
    pool = sale.Pool(ARENA, max_runs=8, precision=precision)
    p, keep = user_prob(st)
    a = pool.admit(cfg, p, steps)
    drain(pool, 4, 1)
    alone = pool.fields(a)
    assert pool.state(a) == ref_state
    # in a mix: other runs of uneven sizes and step counts admitted before and after it
    pool2 = sale.Pool(ARENA, max_runs=8, precision=precision)
    others = []
    for k, m in enumerate(((64, 5, 3), (7, 7, 7), (20, 48, 2))):
        c2 = sale.make_config(*m, hi=(1.0, 1.0, 1.0), t_end=100.0, precision=precision)
        p2, k2 = user_prob(random_state(*m, seed=100 + k))
        others.append(pool2.admit(c2, p2, 3 + 5 * k))
        if k == 0:
            p, keep = user_prob(st)
            b = pool2.admit(cfg, p, steps)
    drain(pool2, 2, 4)
    mix = pool2.fields(b)
    assert pool2.state(b) == ref_state
    for k in FIELDS:
        assert np.array_equal(alone[k], ref[k]), k
        assert np.array_equal(mix[k], ref[k]), k


def test_pool_slots_and_arena_are_reused_and_admission_refuses_when_full():
    say("pool reuse / EBUSY")
    cfg = sale.make_config(24, 24, 24, hi=(1.2, 1.2, 1.2), t_end=1.0)
    per_run = sale.sale_workspace_bytes(cfg)
    # room for two runs of this size (plus the header), not three
    pool = sale.Pool(2 * per_run + (1 << 20), max_runs=4)
    a = pool.admit(cfg, sale.sedov_problem(), 5)
    b = pool.admit(cfg, sale.sedov_problem(), 8)
    assert a is not None and b is not None
    assert pool.admit(cfg, sale.sedov_problem(), 5) is None          # arena full
    small = sale.make_config(4, 4, 4, hi=(1.2, 1.2, 1.2), t_end=1.0)
    c = pool.admit(small, sale.sedov_problem(), 3)                    # a small run still fits
    assert c is not None
    d = pool.admit(small, sale.sedov_problem(), 3)
    e = pool.admit(small, sale.sedov_problem(), 3)
    assert d is not None and e is None                                 # 4 slots
    # a run larger than the arena's room for runs can never be admitted: ENOMEM, not EBUSY
    big = sale.make_config(64, 64, 64, hi=(1.2, 1.2, 1.2), t_end=1.0)
    with pytest.raises(sale.SaleError) as err:
        pool.admit(big, sale.sedov_problem(), 3)
    assert err.value.code == sale.SALE_ENOMEM
    done = drain(pool, 3, 4)
    assert sorted(done) == sorted([a, b, c, d])
    ref = pool.fields(a)
    pool.release(a)
    pool.release(c)
    # the freed range takes a new run; its result equals the first run of the same problem
    f = pool.admit(cfg, sale.sedov_problem(), 5)
    assert f is not None
    assert drain(pool, 2, 1) == [f]
    got = pool.fields(f)
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    # finished runs (b, d) were not advanced further
    assert pool.state(b)[1] == 8 and pool.state(d)[1] == 3


def test_pool_flag_stops_only_the_flagged_run():
    say("pool flag isolation")
    # the forced predictor tangle of the single-run error test
    cfg_bad = sale.make_config(3, 3, 3, cfl=0.99, c_quad=0.0, c_lin=0.0, t_end=1.0)
    g = grid_of(cfg_bad)
    s = orc.empty_state(g)
    s.rho[...] = 1.0
    s.e[...] = 1e-8
    for c in (1, 2):
        for b in (1, 2):
            for a in (1, 2):
                s.u[c, b, a] = -10.0 * (2 * (a - 1) - 1)
                s.v[c, b, a] = -10.0 * (2 * (b - 1) - 1)
                s.w[c, b, a] = -10.0 * (2 * (c - 1) - 1)
    cfg_ok = sale.make_config(16, 16, 16, hi=(1.2, 1.2, 1.2), t_end=1.0)
    pool = sale.Pool(ARENA, max_runs=4)
    p, keep = user_prob(s.fields())
    bad = pool.admit(cfg_bad, p, 10)
    good = pool.admit(cfg_ok, sale.sedov_problem(), 10)
    pool.advance(10)
    assert sorted(pool.poll()) == sorted([bad, good])
    assert pool.state(bad)[3] & sale.SALE_FLAG_TANGLE
    t, nstep, _, flags = pool.state(good)
    assert flags == 0 and nstep == 10
    r = sale.SaleRun(cfg_ok, sale.sedov_problem())
    r.step(10)
    ref = r.fields()
    got = pool.fields(good)
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k


def test_pool_end_time_and_step_target():
    say("pool t_end / n_steps")
    cfg = sale.make_config(32, 2, 2, hi=(1.0, 0.0625, 0.0625), t_end=0.05)
    pool = sale.Pool(ARENA, max_runs=4)
    a = pool.admit(cfg, sale.sod_problem(), 1 << 40)      # stops at t_end
    b = pool.admit(cfg, sale.sod_problem(), 0)            # zero steps: done at once
    drain(pool, 7, 2)
    assert pool.state(a)[0] == 0.05
    r = sale.SaleRun(cfg, sale.sod_problem())
    assert r.run() == sale.SALE_DONE
    assert pool.state(a)[:2] == r.state()[:2]
    got, ref = pool.fields(a), r.fields()
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    t, nstep, _, _ = pool.state(b)
    assert t == 0.0 and nstep == 0
