"""The C oracle against an independently written NumPy implementation, and
the whole scheme against exact solutions of the paper's verification flows
(Sod shock tube, Sedov-Taylor blast; Sec. I-D, Fig. 2). CPU only."""
import numpy as np
import pytest

from oracle import mini_oracle
from oracle import oracle as orc
from oracle.exact import SodExact, sedov_radius
from paper_2209_01983_amd.inputs import random_state


def _relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,seed,smooth", [((4, 4, 4), 11, False), ((7, 5, 3), 12, False),
                                            ((16, 16, 16), 13, True), ((1, 6, 2), 14, False)])
def test_c_oracle_matches_numpy_mini_oracle(n, seed, smooth):
    g = orc.Grid(*n, hi=(1.0, 1.3, 0.7), t_end=100.0)
    st = random_state(*n, seed=seed, smooth=smooth)
    s = orc.State(**{k: v.copy() for k, v in st.items()})
    o = orc.Oracle(g)
    r, e, u, v, w, t = st["rho"], st["e"], st["u"], st["v"], st["w"], 0.0
    for _ in range(20):
        rc, dt = o.step(s)
        assert rc == orc.OK
        r, e, u, v, w, t, dt2 = mini_oracle.step(g, r, e, u, v, w, t)
        assert dt == pytest.approx(dt2, rel=1e-13)
        for name, a, b in (("rho", s.rho, r), ("e", s.e, e), ("u", s.u, u), ("v", s.v, v), ("w", s.w, w)):
            if np.abs(b).max() == 0:
                assert np.all(a == 0), name
            else:
                assert _relmax(a, b) <= 1e-13, name


def test_c_oracle_matches_mini_oracle_on_sedov():
    g = orc.Grid(8, 8, 8, hi=(1.2, 1.2, 1.2))
    s = orc.sedov(g)
    r, e, u, v, w, t = s.rho.copy(), s.e.copy(), s.u.copy(), s.v.copy(), s.w.copy(), 0.0
    o = orc.Oracle(g)
    for _ in range(15):
        assert o.step(s)[0] == orc.OK
        r, e, u, v, w, t, _ = mini_oracle.step(g, r, e, u, v, w, t)
    for a, b in ((s.rho, r), (s.e, e), (s.u, u), (s.v, v), (s.w, w)):
        assert _relmax(a, b) <= 1e-13


# ---------------------------------------------------------------------------
# Sod: L1 error against the exact Riemann solution converges under refinement
# ---------------------------------------------------------------------------
def sod_l1(nx):
    g = orc.Grid(nx, 1, 1, hi=(1.0, 1.0 / nx, 1.0 / nx), t_end=0.2)
    s = orc.sod(g)
    rc, _ = orc.Oracle(g).run(s)
    assert rc == orc.DONE and s.t == 0.2
    xc = (np.arange(nx) + 0.5) / nx
    xn = np.arange(nx + 1) / nx
    ex = SodExact()
    r_ex, _, p_ex, e_ex = ex.sample(xc, 0.2)
    _, u_ex, _, _ = ex.sample(xn, 0.2)
    rho, e = s.rho[0, 0], s.e[0, 0]
    p = 0.4 * rho * e
    u = s.u[0, 0]
    l1 = lambda a, b, h: np.sum(np.abs(a - b)) * h
    return {"rho": l1(rho, r_ex, 1 / nx), "e": l1(e, e_ex, 1 / nx), "p": l1(p, p_ex, 1 / nx),
            "u": l1(u, u_ex, 1 / nx)}


def test_sod_l1_converges_to_exact_solution():
    ns = [64, 128, 256, 512]
    errs = [sod_l1(n) for n in ns]
    for f in ("rho", "u", "p", "e"):
        seq = [er[f] for er in errs]
        assert all(b < a for a, b in zip(seq, seq[1:])), (f, seq)
        order = np.log2(seq[0] / seq[-1]) / np.log2(ns[-1] / ns[0])
        assert order >= 0.5, (f, seq, order)
    assert errs[0]["rho"] < 0.03


def test_sod_config_mesh_matches_exact_solution():
    """The 64 x 4 x 4 tube to t = 0.2: every row has the 1D error level."""
    g = orc.Grid(64, 4, 4, hi=(1.0, 0.0625, 0.0625), t_end=0.2)
    s = orc.sod(g)
    assert orc.Oracle(g).run(s)[0] == orc.DONE
    xc = (np.arange(64) + 0.5) / 64
    r_ex, _, _, _ = SodExact().sample(xc, 0.2)
    l1 = np.abs(s.rho - r_ex[None, None, :]).sum(axis=-1) / 64
    assert l1.max() == pytest.approx(sod_l1(64)["rho"], rel=1e-9)


# ---------------------------------------------------------------------------
# Sedov: shock radius against the self-similar solution
# ---------------------------------------------------------------------------
def sedov_shock_radius(n, t_end=1.0):
    g = orc.Grid(n, n, n, hi=(1.2, 1.2, 1.2), t_end=t_end)
    s = orc.sedov(g)
    rc, steps = orc.Oracle(g).run(s)
    assert rc == orc.DONE
    m0, E0 = orc.Oracle(g).totals(orc.sedov(g))
    m1, E1 = orc.Oracle(g).totals(s)
    assert abs(m1 - m0) / m0 < 1e-13 and abs(E1 - E0) / E0 < 1e-12
    r = (np.arange(n) + 0.5) * 1.2 / n
    radii = [r[np.argmax(s.rho[0, 0, :])], r[np.argmax(s.rho[0, :, 0])], r[np.argmax(s.rho[:, 0, 0])],
             r[np.argmax(np.einsum("iii->i", s.rho))] * np.sqrt(3.0)]
    return radii, steps


def test_sedov_shock_radius_32():
    radii, _ = sedov_shock_radius(32)
    R = sedov_radius(1.0)  # E = 8 x 0.125 in full space
    assert abs(np.mean(radii) - R) / R <= 0.04
    assert radii[0] == radii[1] == radii[2]


@pytest.mark.slow
def test_sedov_shock_radius_refines_64():
    R = sedov_radius(1.0)
    r32, _ = sedov_shock_radius(32)
    r64, _ = sedov_shock_radius(64)
    assert abs(np.mean(r64) - R) / R <= 0.04
    # the diagonal (most diffused) estimate improves with refinement
    assert abs(r64[3] - R) <= abs(r32[3] - R) + 1.2 / 64
