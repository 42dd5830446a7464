"""Noh implosion (Sec. I-D lists it among the problems ScalSALE solves, in 1D,
2D and 3D): the closed-form solution pinned to the Rankine-Hugoniot
conditions and the continuity equation, the oracle's initial state to its
definition, and the oracle's runs to the closed form (planar: accuracy and
first-order convergence; cylindrical and spherical: mass balance inside a
radius, converging, and exact symmetry), plus the C oracle against the
independent NumPy implementation on a convergent flow. CPU only."""
import numpy as np
import pytest

from oracle import mini_oracle
from oracle import oracle as orc
from oracle.exact import NohExact

G53 = 5.0 / 3.0


# ---------------------------------------------------------------------------
# the closed form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [1, 2, 3])
@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.4])
def test_noh_exact_satisfies_rankine_hugoniot(dims, gamma):
    ex = NohExact(gamma=gamma, u0=1.3, rho0=0.7, dims=dims)
    t = 0.8
    rs = ex.shock_radius(t)
    (r1, u1, p1, e1), (r2, u2, p2, e2) = [tuple(np.ravel(a)[0] for a in ex.sample(np.array([x]), t))
                                          for x in (rs * (1 + 1e-12), rs * (1 - 1e-12))]
    D = ex.D  # the shock moves outward (+r), the gas ahead of it inward
    w1, w2 = u1 - D, u2 - D  # speeds relative to the shock
    assert r1 * w1 == pytest.approx(r2 * w2, rel=1e-9)
    assert r1 * w1 * w1 + p1 == pytest.approx(r2 * w2 * w2 + p2, rel=1e-9)
    h1 = e1 + p1 / r1 + 0.5 * w1 * w1
    h2 = e2 + p2 / r2 + 0.5 * w2 * w2
    assert h1 == pytest.approx(h2, rel=1e-9)
    # ideal-gas pressure and rest behind the shock
    assert p2 == pytest.approx((gamma - 1) * r2 * e2) and u2 == 0.0


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_noh_exact_preshock_obeys_continuity(dims):
    """d(rho)/dt + r^(1-n) d(r^(n-1) rho u)/dr = 0 ahead of the shock
    (central differences)."""
    ex = NohExact(gamma=G53, u0=1.0, rho0=1.0, dims=dims)
    r = np.linspace(0.4, 2.0, 17)
    t, d = 0.6, 1e-5
    rho_t = (ex.sample(r, t + d)[0] - ex.sample(r, t - d)[0]) / (2 * d)
    flux = lambda x: x ** (dims - 1) * ex.sample(x, t)[0] * ex.sample(x, t)[1]
    div = (flux(r + d) - flux(r - d)) / (2 * d) / r ** (dims - 1)
    assert np.max(np.abs(rho_t + div)) < 1e-6


# ---------------------------------------------------------------------------
# the oracle's initial state
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [1, 2, 3])
def test_noh_initial_state(dims):
    g = orc.Grid(6, 5, 4, hi=(1.0, 0.9, 0.7), gamma=G53)
    u0 = 1.7
    s = orc.noh(g, rho0=2.0, p0=3e-6, u0=u0, dims=dims)
    assert np.all(s.rho == 2.0)
    assert np.allclose(s.e, 3e-6 / ((G53 - 1) * 2.0), rtol=1e-15)
    dx, dy, dz = g.spacing
    K, J, I = np.meshgrid(np.arange(g.nz + 1), np.arange(g.ny + 1), np.arange(g.nx + 1), indexing="ij")
    r = np.stack([I * dx, J * dy * (dims >= 2), K * dz * (dims >= 3)])
    vel = np.stack([s.u, s.v, s.w])
    walls = [(I == 0) | (I == g.nx), (J == 0) | (J == g.ny), (K == 0) | (K == g.nz)]
    for a in range(3):
        assert np.all(vel[a][walls[a]] == 0.0)  # reflective walls
        if a >= dims:
            assert np.all(vel[a] == 0.0)
    inner = ~(walls[0] | walls[1] | walls[2])
    rr = np.sqrt((r ** 2).sum(axis=0))
    # away from the walls: speed u0, pointing at the corner lo
    speed = np.sqrt((vel ** 2).sum(axis=0))
    assert np.allclose(speed[inner], u0, rtol=1e-14)
    cross = np.cross(vel[:, inner].T, r[:, inner].T)
    assert np.max(np.abs(cross)) < 1e-13
    assert np.all((vel[:, inner] * r[:, inner]).sum(axis=0) < 0)
    # on a wall only the normal component is dropped
    on_x = walls[0] & ~walls[1] & ~walls[2] & (I == g.nx)
    if dims >= 2:
        assert np.allclose(s.v[on_x], -u0 * r[1][on_x] / rr[on_x], rtol=1e-14)


def test_noh_rejects_bad_dims():
    with pytest.raises(ValueError):
        orc.noh(orc.Grid(4, 4, 4), dims=4)


# ---------------------------------------------------------------------------
# planar Noh: accuracy and first-order convergence
# ---------------------------------------------------------------------------
def planar_noh(n, t=0.6):
    g = orc.Grid(n, 1, 1, hi=(1.0, 1.0 / n, 1.0 / n), gamma=G53, t_end=t)
    s = orc.noh(g, p0=1e-6, dims=1)
    rc, _ = orc.Oracle(g).run(s)
    assert rc == orc.DONE and s.t == t
    return s


def test_planar_noh_matches_closed_form():
    """200 cells to t = 0.6: the shock stands at 0.2 and the gas behind it is
    at rest with rho = 4 and e = 1/2 (gamma = 5/3); the wall-heating dip of
    the first few cells next to the wall (an artefact of artificial-viscosity
    schemes, Noh 1987) is left out."""
    n, t = 200, 0.6
    s = planar_noh(n, t)
    ex = NohExact(G53, dims=1)
    x = (np.arange(n) + 0.5) / n
    xn = np.arange(n + 1) / n
    rho, e, u = s.rho[0, 0], s.e[0, 0], s.u[0, 0]
    plateau = (x > 0.05) & (x < 0.17)
    assert np.max(np.abs(rho[plateau] / ex.rho_post - 1)) < 2e-3
    assert np.max(np.abs(e[plateau] / ex.e_post - 1)) < 2e-3
    assert np.max(np.abs(u[(xn > 0.05) & (xn < 0.17)])) < 1e-3
    # ahead of the shock, short of the smeared rarefaction that the closed
    # wall at x = 1 sends in
    pre = (x > 0.22) & (x < 0.25)
    assert np.max(np.abs(rho[pre] - 1.0)) < 1.5e-2
    assert np.max(np.abs(u[(xn > 0.22) & (xn < 0.25)] + 1.0)) < 1.5e-2
    i = int(np.argmax(rho < 2.5))
    xs = x[i - 1] + (rho[i - 1] - 2.5) / (rho[i - 1] - rho[i]) * (x[i] - x[i - 1])
    assert abs(xs - ex.shock_radius(t)) < 1.0 / n


def test_planar_noh_l1_converges():
    ex = NohExact(G53, dims=1)
    errs = []
    for n in (100, 200, 400):
        s = planar_noh(n)
        x = (np.arange(n) + 0.5) / n
        m = x < 0.35
        errs.append(np.sum(np.abs(s.rho[0, 0][m] - ex.sample(x[m], 0.6)[0])) / n)
    assert errs[0] > errs[1] > errs[2]
    rate = np.log2(errs[0] / errs[2]) / 2
    assert rate > 0.85, (errs, rate)


# ---------------------------------------------------------------------------
# cylindrical and spherical Noh: mass balance, convergence, symmetry
# ---------------------------------------------------------------------------
def multi_d_noh(n, dims, t=0.6):
    nz = n if dims == 3 else 1
    g = orc.Grid(n, n, nz, hi=(1.0, 1.0, nz / n), gamma=G53, t_end=t)
    s = orc.noh(g, p0=1e-6, dims=dims)
    rc, _ = orc.Oracle(g).run(s)
    assert rc == orc.DONE and s.t == t
    return g, s


def mass_inside(g, s, dims, R, t):
    """(computed, closed-form) mass of the cells whose centres lie within R
    of the corner; the closed form is the initial mass of that region plus
    the inflow through the arc/sphere, rescaled by the cells' share of the
    continuous region's volume."""
    h = g.spacing[0]
    c = (np.arange(g.nx) + 0.5) * h
    z = (np.arange(g.nz) + 0.5) * g.spacing[2] if dims == 3 else np.zeros(1)
    Z, Y, X = np.meshgrid(z, c, c, indexing="ij")
    inside = np.sqrt(X ** 2 + Y ** 2 + Z ** 2) < R
    V0 = h * h * g.spacing[2]
    got = s.rho[inside].sum() * V0
    if dims == 2:
        region = np.pi * R * R / 4 * g.spacing[2]
        inflow = np.pi / 2 * R * (t + t * t / (2 * R)) * g.spacing[2]
    else:
        region = np.pi * R ** 3 / 6
        inflow = np.pi / 2 * R * R * (t + t * t / R + t ** 3 / (3 * R * R))
    share = inside.sum() * V0 / region
    return got, (region + inflow) * share


def test_cylindrical_noh_mass_balance_converges():
    errs = []
    for n in (64, 128):
        g, s = multi_d_noh(n, 2)
        got, want = mass_inside(g, s, 2, 0.35, 0.6)
        errs.append(abs(got / want - 1))
        assert np.max(np.abs(s.rho - s.rho.transpose(0, 2, 1))) <= 1e-12 * s.rho.max()
    assert errs[1] < errs[0] and errs[1] < 0.012, errs
    # the preshock density follows (1 + t/r) at the finer resolution
    c = (np.arange(128) + 0.5) / 128
    Y, X = np.meshgrid(c, c, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2)
    pre = (r > 0.26) & (r < 0.3)
    exact = NohExact(G53, dims=2).sample(r[pre], 0.6)[0]
    assert np.mean(np.abs(s.rho[0][pre] / exact - 1)) < 0.05


def test_spherical_noh_mass_balance_converges_and_is_symmetric():
    """The first-order Eulerian scheme resolves the 3D implosion poorly at
    these sizes (the shock is 6-10 cells from the corner); what is pinned is
    that the mass balance inside r = 0.35 improves under refinement and that
    the solution is symmetric under every exchange of axes."""
    errs = []
    for n in (32, 48):
        g, s = multi_d_noh(n, 3)
        got, want = mass_inside(g, s, 3, 0.35, 0.6)
        errs.append(abs(got / want - 1))
        top = s.rho.max()
        for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
            assert np.max(np.abs(s.rho - s.rho.transpose(perm))) <= 1e-12 * top
        assert np.max(np.abs(s.u - s.v.transpose(0, 2, 1))) <= 1e-12
    assert errs[1] < 0.6 * errs[0], errs


def test_c_oracle_matches_mini_oracle_on_noh():
    g = orc.Grid(9, 7, 8, hi=(1.0, 0.8, 0.9), gamma=G53, t_end=10.0)
    s = orc.noh(g, p0=1e-6, dims=3)
    r, e, u, v, w, t = s.rho.copy(), s.e.copy(), s.u.copy(), s.v.copy(), s.w.copy(), 0.0
    o = orc.Oracle(g)
    for _ in range(12):
        assert o.step(s)[0] == orc.OK
        r, e, u, v, w, t, _ = mini_oracle.step(g, r, e, u, v, w, t)
    for a, b in ((s.rho, r), (s.e, e), (s.u, u), (s.v, v), (s.w, w)):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
