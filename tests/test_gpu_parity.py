"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP64): per field, max |gpu - oracle| / max |oracle| <= 1e-12 after every
step compared; fields the oracle has identically zero must be zero. Sizes:
small meshes spanning several thread blocks with ragged tails (whole
trajectories), the paper's flows at their configured sizes, and the 320^3
Sedov mesh in the benchmark's launch configuration (one full step from a
developed state). Properties that hold at any size (conservation, symmetry,
determinism, restart) are checked on the GPU runs themselves.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle.exact import sedov_radius
from paper_2209_01983_amd import sale
from paper_2209_01983_amd.inputs import random_state

from parity import FIELDS, TOL64, assert_parity, errors, grid_of, oracle_state, say  # noqa: E402

pytestmark = pytest.mark.gpu


def sod_cfg():
    return sale.make_config(64, 4, 4, hi=(1.0, 0.0625, 0.0625), t_end=0.2)


def sedov_cfg(n, t_end=1.0):
    return sale.make_config(n, n, n, hi=(1.2, 1.2, 1.2), t_end=t_end)


def user_run(cfg, st, t0=0.0, step0=0):
    p, keep = sale.user_problem(st["rho"], st["e"], st["u"], st["v"], st["w"], t0=t0, step0=step0)
    return sale.SaleRun(cfg, p, keepalive=keep)


def test_sod_whole_trajectory_matches_oracle():
    cfg = sod_cfg()
    say("sod 64x4x4 trajectory")
    r = sale.SaleRun(cfg, sale.sod_problem())
    g = grid_of(cfg)
    s = orc.sod(g)
    o = orc.Oracle(g)
    assert_parity(r.fields(), s, what="init")
    worst = {k: 0.0 for k in FIELDS}
    n = 0
    while True:
        rc, dt = o.step(s)
        if rc == orc.DONE:
            break
        assert rc == orc.OK
        r.step()
        n += 1
        err = assert_parity(r.fields(), s, what=f"step {n}")
        worst = {k: max(worst[k], err[k]) for k in FIELDS}
        t, steps, _, flags = r.state()
        assert flags == 0 and steps == n
        assert t == pytest.approx(s.t, rel=1e-14)
    assert r.run() == sale.SALE_DONE
    assert r.state()[0] == 0.2 and n == s.step
    say("sod worst per-field error", worst)


@pytest.mark.parametrize("n,seed", [((37, 29, 23), 1), ((65, 3, 2), 2), ((1, 1, 1), 3), ((1, 7, 1), 4),
                                    ((5, 1, 9), 5), ((130, 17, 5), 6)])
def test_random_states_on_ragged_meshes(n, seed):
    say("random", n, seed)
    cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0)
    st = random_state(*n, seed=seed)
    r = user_run(cfg, st)
    s = oracle_state(st)
    o = orc.Oracle(grid_of(cfg))
    for step in range(6):
        assert o.step(s)[0] == orc.OK
        r.step()
        assert_parity(r.fields(), s, what=f"{n} step {step}")


def test_device_and_host_user_arrays_agree_bitwise():
    import torch
    say("user arrays device vs host")
    n = (20, 9, 14)
    cfg = sale.make_config(*n, t_end=100.0)
    st = random_state(*n, seed=21, smooth=True)
    a = user_run(cfg, st)
    dev = {k: torch.from_numpy(v).cuda() for k, v in st.items()}
    p, keep = sale.user_problem(dev["rho"], dev["e"], dev["u"], dev["v"], dev["w"])
    b = sale.SaleRun(cfg, p, keepalive=keep)
    a.step(5)
    b.step(5)
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        assert np.array_equal(fa[k], fb[k]), k


def test_sedov_48_trajectory_matches_oracle():
    say("sedov 48^3 trajectory")
    cfg = sedov_cfg(48)
    r = sale.SaleRun(cfg, sale.sedov_problem())
    g = grid_of(cfg)
    s = orc.sedov(g)
    o = orc.Oracle(g)
    for step in range(80):
        assert o.step(s)[0] == orc.OK
        r.step()
        if step % 4 == 3:
            assert_parity(r.fields(), s, what=f"step {step}")


def _single_step_check(r, cfg, o, what):
    """One oracle step from the GPU's current state against one GPU step."""
    t, steps, _, _ = r.state()
    s = oracle_state(r.fields(), t=t, step=steps)
    rc, _ = o.step(s)
    assert rc == orc.OK, what
    r.step()
    err = assert_parity(r.fields(), s, what=what)
    assert r.state()[0] == pytest.approx(s.t, rel=1e-14)
    return err


def test_sedov_128_full_run_single_step_parity_and_physics():
    """Sedov 128^3 to t = 1: single-step parity from the GPU's states at steps
    0, 1, 10, 100 and the last step, mass/energy conservation, symmetry and
    the shock radius."""
    cfg = sedov_cfg(128)
    g = grid_of(cfg)
    o = orc.Oracle(g)
    # first: how many steps to t = 1
    say("sedov 128^3 full run")
    full = sale.SaleRun(cfg, sale.sedov_problem())
    m0, E0 = full.totals()
    m_or, E_or = o.totals(orc.sedov(g))
    assert m0 == pytest.approx(m_or, rel=1e-13) and E0 == pytest.approx(E_or, rel=1e-13)
    assert full.run() == sale.SALE_DONE
    t, nsteps, _, flags = full.state()
    assert t == 1.0 and flags == 0
    m1, E1 = full.totals()
    assert abs(m1 - m0) / m0 <= 1e-13 and abs(E1 - E0) / E0 <= 1e-12
    fs = full.fields()
    for f in (fs["rho"], fs["e"]):
        sc = np.abs(f).max()
        for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
            assert np.abs(f - f.transpose(perm)).max() <= 1e-13 * sc
    rr = (np.arange(128) + 0.5) * 1.2 / 128
    radii = [rr[np.argmax(fs["rho"][0, 0, :])], rr[np.argmax(fs["rho"][0, :, 0])],
             rr[np.argmax(fs["rho"][:, 0, 0])], rr[np.argmax(np.einsum("iii->i", fs["rho"]))] * np.sqrt(3)]
    R = sedov_radius(1.0)
    say("sedov 128 steps", nsteps, "radii", radii, "exact", R)
    assert abs(np.mean(radii) - R) / R <= 0.04
    assert fs["e"].min() > 0
    del full
    # single steps from states along the same trajectory
    r = sale.SaleRun(cfg, sale.sedov_problem())
    done = 0
    for at in (0, 1, 10, 100, nsteps - 1):
        if at > done:
            assert r.run(max_steps=at - done) == sale.SALE_OK
            done = at
        say("sedov 128 single step at", at)
        _single_step_check(r, cfg, o, f"step {at}")
        done += 1


def test_sedov_320_single_step_parity_bench_configuration():
    """The benchmark's mesh and launch configuration: one oracle step on the
    full 320^3 mesh from a developed GPU state."""
    cfg = sedov_cfg(320)
    say("sedov 320^3: 30 GPU steps")
    r = sale.SaleRun(cfg, sale.sedov_problem())
    assert r.run(max_steps=30) == sale.SALE_OK
    say("sedov 320^3: oracle workspace")
    o = orc.Oracle(grid_of(cfg))
    say("sedov 320^3: single step")
    err = _single_step_check(r, cfg, o, "320^3")
    say("320^3 errors", err)


def test_determinism_and_restart_are_bitwise():
    cfg = sedov_cfg(40, t_end=10.0)
    say("determinism / restart")
    a = sale.SaleRun(cfg, sale.sedov_problem())
    a.step(40)
    b = sale.SaleRun(cfg, sale.sedov_problem())
    b.step(40)
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        assert np.array_equal(fa[k], fb[k]), k
    assert a.state() == b.state()
    c = sale.SaleRun(cfg, sale.sedov_problem())
    c.step(15)
    t, steps, _, _ = c.state()
    d = user_run(cfg, c.fields(), t0=t, step0=steps)
    d.step(25)
    fd = d.fields()
    for k in FIELDS:
        assert np.array_equal(fa[k], fd[k]), k
    assert d.state()[:2] == a.state()[:2]


def test_quiescent_fixed_point_and_untouched_background():
    say("fixed point")
    cfg = sale.make_config(33, 17, 9, t_end=1e6)
    st = {"rho": np.full((9, 17, 33), 1.37), "e": np.full((9, 17, 33), 0.291),
          "u": np.zeros((10, 18, 34)), "v": np.zeros((10, 18, 34)), "w": np.zeros((10, 18, 34))}
    r = user_run(cfg, st)
    r.step(10)
    f = r.fields()
    for k in FIELDS:
        assert np.array_equal(f[k], st[k]), k
    cfg = sedov_cfg(64)
    r = sale.SaleRun(cfg, sale.sedov_problem())
    f0 = r.fields()
    r.step(3)
    f = r.fields()
    kk, jj, ii = np.indices((64, 64, 64))
    far = np.maximum(np.maximum(ii, jj), kk) >= 13
    assert np.array_equal(f["rho"][far], f0["rho"][far]) and np.array_equal(f["e"][far], f0["e"][far])


def test_derived_fields_and_totals():
    say("derived fields")
    n = (24, 11, 7)
    cfg = sale.make_config(*n, t_end=100.0)
    st = random_state(*n, seed=31)
    r = user_run(cfg, st)
    r.step(3)
    g = grid_of(cfg)
    f = r.fields(("rho", "e", "p", "q", "u", "v", "w"))
    s = oracle_state(f)
    o = orc.Oracle(g)
    p, q = o.derived(s)
    assert np.abs(f["p"] - p).max() <= 1e-15 * np.abs(p).max()
    assert np.abs(f["q"] - q).max() <= 1e-13 * np.abs(q).max()
    m, E = r.totals()
    mo, Eo = o.totals(s)
    assert m == pytest.approx(mo, rel=1e-14) and E == pytest.approx(Eo, rel=1e-14)
    dev = r.fields(("rho", "u"), on_device=True)
    assert np.array_equal(dev["rho"].cpu().numpy(), f["rho"]) and np.array_equal(dev["u"].cpu().numpy(), f["u"])


def test_error_codes_match_oracle():
    import torch
    say("error codes")
    # forced predictor tangle: CFL 0.99, no viscosity, converging centre cell
    cfg = sale.make_config(3, 3, 3, cfl=0.99, c_quad=0.0, c_lin=0.0, t_end=1.0)
    g = grid_of(cfg)
    s = orc.empty_state(g)
    s.rho[...] = 1.0
    s.e[...] = 1e-8
    for c in (1, 2):
        for b in (1, 2):
            for a in (1, 2):
                s.u[c, b, a] = -10.0 * (2 * (a - 1) - 1)
                s.v[c, b, a] = -10.0 * (2 * (b - 1) - 1)
                s.w[c, b, a] = -10.0 * (2 * (c - 1) - 1)
    assert orc.Oracle(g).step(s.copy())[0] == orc.ETANGLE
    r = user_run(cfg, s.fields())
    r.step()
    rc, flags = r.status()
    assert rc == sale.SALE_ETANGLE and flags & sale.SALE_FLAG_TANGLE
    assert r.run() == sale.SALE_ETANGLE
    # device arrays with a NaN / a negative energy: flagged on the device
    n = (6, 5, 4)
    cfg = sale.make_config(*n, t_end=1.0)
    for field, val in (("e", float("nan")), ("e", -1.0), ("rho", 0.0), ("u", float("inf"))):
        st = random_state(*n, seed=41)
        # an interior cell / node (wall-normal velocities are reset at init)
        st[field][1, 1, 1] = val
        dev = {k: torch.from_numpy(v).cuda() for k, v in st.items()}
        p, keep = sale.user_problem(dev["rho"], dev["e"], dev["u"], dev["v"], dev["w"])
        r = sale.SaleRun(cfg, p, keepalive=keep)
        rc, flags = r.status()
        assert rc == sale.SALE_ENUMERIC and flags & sale.SALE_FLAG_NUMERIC, (field, val)
        st_h = oracle_state(st)
        assert orc.Oracle(grid_of(cfg)).step(st_h)[0] == orc.ENUMERIC, (field, val)
    # done: steps after t_end change nothing
    cfg = sale.make_config(16, 2, 2, hi=(1.0, 0.125, 0.125), t_end=0.05)
    r = sale.SaleRun(cfg, sale.sod_problem())
    assert r.run() == sale.SALE_DONE
    f0 = r.fields()
    st0 = r.state()
    r.step(3)
    f1 = r.fields()
    assert r.state() == st0 and st0[0] == 0.05
    for k in FIELDS:
        assert np.array_equal(f0[k], f1[k])
    # a later end time continues the run
    assert r.run(t_end=0.1) == sale.SALE_DONE and r.state()[0] == 0.1


# ---------------------------------------------------------------------------
# MIXED32: FP32 bulk arithmetic, FP64 geometry / dt / totals
# ---------------------------------------------------------------------------
# Stated error bars (relative to the field's scale, as above): one step from a
# smooth random state <= 5e-6 per field; the Sod tube to t = 0.2 <= 5e-6 vs the
# FP64 oracle; mass and energy drift of a Sedov run <= 1e-6 / 1e-5.
TOL32_STEP = 5e-6


def mixed_cfg(*a, **k):
    return sale.make_config(*a, precision=sale.SALE_MIXED32, **k)


def test_mixed32_single_steps_vs_fp64_oracle():
    n = (37, 29, 23)
    cfg = mixed_cfg(*n, hi=(1.0, 0.8, 1.3), t_end=100.0)
    st = random_state(*n, seed=1, smooth=True)
    r = user_run(cfg, st)
    s = oracle_state(st)
    o = orc.Oracle(grid_of(cfg))
    for step in range(5):
        assert o.step(s)[0] == orc.OK
        r.step()
        err = errors(r.fields(), s)
        assert max(err.values()) <= TOL32_STEP, (step, err)
    say("mixed32 5-step errors", err)


def test_mixed32_sedov_320_single_step_vs_fp64_oracle():
    """MIXED32 in the benchmark's configuration: the full 320^3 Sedov mesh,
    one GPU step from the MIXED32 run's developed state against the FP64
    oracle's step from the same (widened) state, at the single-step bar."""
    cfg = mixed_cfg(320, 320, 320, hi=(1.2, 1.2, 1.2), t_end=1.0)
    say("mixed32 sedov 320^3: 30 GPU steps")
    r = sale.SaleRun(cfg, sale.sedov_problem())
    assert r.run(max_steps=30) == sale.SALE_OK
    t, steps, _, _ = r.state()
    s = oracle_state(r.fields(), t=t, step=steps)
    assert orc.Oracle(grid_of(cfg)).step(s)[0] == orc.OK
    r.step()
    err = errors(r.fields(), s)
    say("mixed32 320^3 errors", err)
    assert max(err.values()) <= TOL32_STEP, err
    assert r.state()[0] == pytest.approx(s.t, rel=1e-6)
    r.close()


def test_mixed32_sod_tube_vs_fp64_oracle():
    cfg = mixed_cfg(64, 4, 4, hi=(1.0, 0.0625, 0.0625), t_end=0.2)
    r = sale.SaleRun(cfg, sale.sod_problem())
    assert r.run() == sale.SALE_DONE
    g = grid_of(cfg)
    s = orc.sod(g)
    assert orc.Oracle(g).run(s)[0] == orc.DONE
    t, steps, _, flags = r.state()
    assert t == 0.2 and flags == 0 and steps == s.step
    err = errors(r.fields(), s)
    say("mixed32 sod errors", err)
    assert max(err.values()) <= 5e-6
    # storage type export is float32 and equals the widened export
    f32 = np.empty((4, 4, 64), dtype=np.float32)
    assert sale.sale_fields(r.ctx, sale.SALE_F_RHO, [f32.ctypes.data], 0, 0) == sale.SALE_OK
    assert np.array_equal(f32.astype(np.float64), r.fields(("rho",))["rho"])


def test_mixed32_sedov_conservation_and_agreement_with_fp64():
    out = {}
    for prec in (sale.SALE_FP64, sale.SALE_MIXED32):
        cfg = sale.make_config(48, 48, 48, hi=(1.2, 1.2, 1.2), t_end=0.3, precision=prec)
        r = sale.SaleRun(cfg, sale.sedov_problem())
        m0, E0 = r.totals()
        assert r.run() == sale.SALE_DONE
        m1, E1 = r.totals()
        out[prec] = (r.fields(), (m1 - m0) / m0, (E1 - E0) / E0, r.state()[1])
    f64, dm64, de64, n64 = out[sale.SALE_FP64]
    f32, dm32, de32, n32 = out[sale.SALE_MIXED32]
    assert abs(dm64) <= 1e-13 and abs(de64) <= 1e-12
    assert abs(dm32) <= 1e-6 and abs(de32) <= 1e-5
    assert n32 == n64
    for k in FIELDS:
        l1 = np.abs(f32[k] - f64[k]).sum() / np.abs(f64[k]).sum()
        assert l1 <= 1e-4, (k, l1)
    say("mixed32 sedov48 drift", dm32, de32)


# ---------------------------------------------------------------------------
# step graphs: sale_run replays captured multi-step graphs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_graph_replays_are_bitwise_the_eager_steps(precision):
    say("graph vs eager, precision", precision)
    te = 0.4
    cfg = sale.make_config(40, 36, 33, hi=(1.2, 1.08, 0.99), t_end=te, precision=precision)
    # eager: one step at a time until t_end
    e = sale.SaleRun(cfg, sale.sedov_problem())
    n = 0
    while e.state()[0] < te:
        e.step()
        n += 1
    assert n > 260, n          # several graph replays of the run below
    # graph path (a context captures its step graph after 128 steps run through
    # sale_run), in pieces with eager work and reads between the replays
    g = sale.SaleRun(cfg, sale.sedov_problem())
    assert g.run(max_steps=141) == sale.SALE_OK      # single steps only
    mid = g.fields()
    g.step(3)
    assert g.run(max_steps=61) == sale.SALE_OK       # graphs and single steps, odd count
    assert g.run() == sale.SALE_DONE
    assert g.state()[:2] == e.state()[:2] and g.state()[1] == n
    ref, got = e.fields(), g.fields()
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    # the replays past t_end changed nothing
    assert g.run(t_end=te, max_steps=16) == sale.SALE_DONE
    again = g.fields()
    for k in FIELDS:
        assert np.array_equal(again[k], ref[k]), k
    # the intermediate read came from a consistent state
    h = sale.SaleRun(cfg, sale.sedov_problem())
    h.step(141)
    hf = h.fields()
    for k in FIELDS:
        assert np.array_equal(hf[k], mid[k]), k


# ---------------------------------------------------------------------------
# launch shapes and the autotuner
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_every_launch_shape_gives_the_same_bits(precision):
    n = (70, 37, 23)
    say("launch shapes", n, precision)
    cfg = sale.make_config(*n, hi=(1.0, 0.8, 1.3), t_end=100.0, precision=precision)
    st = random_state(*n, seed=21)
    ref = None
    for ra, rb, t in ((14, 14, 3072), (7, 7, 3072), (28, 28, 3072), (7, 28, 64), (28, 7, 100000), (14, 28, 1),
                      (14, 7, 500), (14, 14, 0), (7, 14, 0)):
        r = user_run(cfg, st)
        r.set_launch(ra, rb, t)
        r.step(4)
        f = r.fields()
        if ref is None:
            ref = f
            if precision == sale.SALE_FP64:
                s = oracle_state(st)
                o = orc.Oracle(grid_of(cfg))
                for _ in range(4):
                    assert o.step(s)[0] == orc.OK
                assert_parity(f, s, what="default shape")
        else:
            for k in FIELDS:
                assert np.array_equal(f[k], ref[k]), (ra, rb, t, k)
    r = user_run(cfg, st)
    for bad in ((10, 14, 3072), (14, 64, 3072), (16, 14, 3072), (14, 14, -1)):
        assert sale.sale_set_launch(r.ctx, *bad) == sale.SALE_EINVAL


def test_autotuner_picks_a_shape_and_caches_it(tmp_path):
    from paper_2209_01983_amd import tune
    cfg = sale.make_config(48, 48, 48, hi=(1.2, 1.2, 1.2), t_end=1.0)
    path = str(tmp_path / "launch.json")
    best = tune.tune(cfg, steps=2, warmup=1, targets=(1024, 3072), path=path)
    say("tuned", {k: v for k, v in best.items() if k != "candidates"})
    assert best["rows_a"] in tune.ROWS and best["rows_b"] in tune.ROWS and best["target"] in (1024, 3072)
    assert len(best["candidates"]) == 6
    r = sale.SaleRun(cfg, sale.sedov_problem())
    assert tune.apply(r, path=path) == {"rows_a": best["rows_a"], "rows_b": best["rows_b"],
                                        "target": best["target"]}
    r.step(3)
    q = sale.SaleRun(cfg, sale.sedov_problem())
    q.step(3)
    a, b = r.fields(), q.fields()
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def test_step_timed_advances_like_steps_and_times_each_kernel():
    say("step_timed")
    cfg = sedov_cfg(48, t_end=10.0)
    a = sale.SaleRun(cfg, sale.sedov_problem())
    ms = a.step_timed(7)
    assert len(ms) == 3 and all(x > 0.0 for x in ms), ms
    b = sale.SaleRun(cfg, sale.sedov_problem())
    b.step(7)
    assert a.state() == b.state() and a.state()[1] == 7
    fa, fb = a.fields(), b.fields()
    for k in FIELDS:
        assert np.array_equal(fa[k], fb[k]), k
    assert sale.sale_step_timed(a.ctx, 0)[0] == sale.SALE_EINVAL
