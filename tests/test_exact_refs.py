"""Pins of the exact reference solutions against published values and
mathematical identities (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle.exact import SodExact, riemann_star, sedov_alpha

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def test_sod_star_state_matches_published_table():
    ref = _golden("sod_star_state.txt")
    s = SodExact()
    assert s.pstar == pytest.approx(ref["p_star"], abs=6e-6)
    assert s.ustar == pytest.approx(ref["u_star"], abs=6e-6)
    assert s.rho_starL == pytest.approx(ref["rho_star_L"], abs=6e-6)
    assert s.rho_starR == pytest.approx(ref["rho_star_R"], abs=6e-6)


def test_sod_rankine_hugoniot_across_right_shock():
    """Mass, momentum and energy fluxes are continuous in the shock frame."""
    g = 1.4
    s = SodExact()
    S = s.SR
    r1, u1, p1 = 0.125, 0.0, 0.1
    r2, u2, p2 = s.rho_starR, s.ustar, s.pstar
    E1 = p1 / (g - 1) + 0.5 * r1 * u1 ** 2
    E2 = p2 / (g - 1) + 0.5 * r2 * u2 ** 2
    assert r2 * (u2 - S) == pytest.approx(r1 * (u1 - S), rel=1e-12)
    assert r2 * u2 * (u2 - S) + p2 == pytest.approx(r1 * u1 * (u1 - S) + p1, rel=1e-12)
    assert (E2 * (u2 - S) + p2 * u2) == pytest.approx(E1 * (u1 - S) + p1 * u1, rel=1e-12)


def test_sod_rarefaction_is_isentropic_and_continuous():
    s = SodExact()
    x = np.linspace(0.27, 0.48, 50)
    rho, u, p, e = s.sample(x, 0.2)
    assert np.allclose(p / rho ** 1.4, 1.0, rtol=1e-12)
    # continuity at the tail: star state
    r, uu, pp, _ = s.sample(np.array([0.5 + 0.2 * s.STL - 1e-12]), 0.2)
    assert r[0] == pytest.approx(s.rho_starL, rel=1e-9)
    assert uu[0] == pytest.approx(s.ustar, rel=1e-9)


def test_riemann_symmetric_collision_has_zero_star_velocity():
    p, u = riemann_star(1.0, 1.0, 1.0, 1.0, -1.0, 1.0)
    assert abs(u) < 1e-13
    assert p > 1.0


def test_sedov_alpha_matches_literature():
    ref = _golden("sedov_alpha.txt")
    a = sedov_alpha(1.4)
    assert a == pytest.approx(ref["alpha_gamma_1.4"], abs=2e-6)
    assert a ** -0.2 == pytest.approx(1.0328, abs=1e-4)


def test_sedov_alpha_insensitive_to_inner_cutoff():
    assert sedov_alpha(1.4, eta_min=1e-4) == pytest.approx(sedov_alpha(1.4, eta_min=1e-7), rel=1e-6)
