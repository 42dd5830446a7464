"""Exact reference solutions used to pin the oracle (test infrastructure).

* Sod shock tube (the paper's shock-tube verification flow, Sec. I-D and
  Fig. 2a): the exact solution of the 1D Riemann problem for an ideal gas,
  written from the textbook construction (Toro, "Riemann Solvers and Numerical
  Methods for Fluid Dynamics", ch. 4): Newton iteration on the pressure
  function f_L(p) + f_R(p) + u_R - u_L = 0, then sampling of the self-similar
  wave pattern x/t.
* Sedov-Taylor blast (Sec. I-C/I-D, Fig. 2b): the energy constant alpha of
  the self-similar point blast, R(t) = (E t^2 / (alpha rho0))^(1/5), obtained
  by integrating the similarity ODEs inward from the strong-shock
  Rankine-Hugoniot state and evaluating the energy integral.
* Noh implosion (Sec. I-D lists it among ScalSALE's problems; Noh, J. Comput.
  Phys. 72, 1987): cold gas streaming at speed u0 toward the origin in
  1, 2 or 3 dimensions, closed form.

Neither part depends on the oracle or on the HIP path.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp


# --------------------------------------------------------------------------
# Sod: exact Riemann solver
# --------------------------------------------------------------------------
def _pressure_function(p, rho_k, p_k, c_k, gamma):
    """f_K(p) and its derivative for one side K (shock if p > p_K, else rarefaction)."""
    if p > p_k:
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        sq = math.sqrt(A / (p + B))
        f = (p - p_k) * sq
        df = sq * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:
        pr = p / p_k
        f = 2.0 * c_k / (gamma - 1.0) * (pr ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho_k * c_k) * pr ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def riemann_star(rhoL, uL, pL, rhoR, uR, pR, gamma=1.4, tol=1e-14):
    """Star-region pressure and velocity of the exact Riemann solution."""
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    du = uR - uL
    # two-rarefaction estimate as the starting guess
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((cL + cR - 0.5 * (gamma - 1.0) * du) / (cL / pL ** z + cR / pR ** z)) ** (1.0 / z)
    for _ in range(100):
        fL, dfL = _pressure_function(p, rhoL, pL, cL, gamma)
        fR, dfR = _pressure_function(p, rhoR, pR, cR, gamma)
        pn = p - (fL + fR + du) / (dfL + dfR)
        pn = max(pn, tol)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _pressure_function(p, rhoL, pL, cL, gamma)
    fR, _ = _pressure_function(p, rhoR, pR, cR, gamma)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


class SodExact:
    """Exact solution of a 1D Riemann problem with the initial jump at x0."""

    def __init__(self, rhoL=1.0, uL=0.0, pL=1.0, rhoR=0.125, uR=0.0, pR=0.1, gamma=1.4, x0=0.5):
        self.s = (rhoL, uL, pL, rhoR, uR, pR)
        self.g = gamma
        self.x0 = x0
        self.pstar, self.ustar = riemann_star(rhoL, uL, pL, rhoR, uR, pR, gamma)
        g = gamma
        ps, us = self.pstar, self.ustar
        # left wave
        cL = math.sqrt(g * pL / rhoL)
        if ps > pL:
            self.rho_starL = rhoL * ((ps / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pL + 1))
            self.SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
            self.left_shock = True
        else:
            self.rho_starL = rhoL * (ps / pL) ** (1.0 / g)
            self.left_shock = False
            cstarL = cL * (ps / pL) ** ((g - 1) / (2 * g))
            self.SHL = uL - cL
            self.STL = us - cstarL
        # right wave
        cR = math.sqrt(g * pR / rhoR)
        if ps > pR:
            self.rho_starR = rhoR * ((ps / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pR + 1))
            self.SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
            self.right_shock = True
        else:
            self.rho_starR = rhoR * (ps / pR) ** (1.0 / g)
            self.right_shock = False
            cstarR = cR * (ps / pR) ** ((g - 1) / (2 * g))
            self.SHR = uR + cR
            self.STR = us + cstarR

    def sample(self, x, t):
        """(rho, u, p, e) at positions x (array) and time t > 0."""
        rhoL, uL, pL, rhoR, uR, pR = self.s
        g = self.g
        xi = (np.asarray(x, dtype=np.float64) - self.x0) / t
        rho = np.empty_like(xi)
        u = np.empty_like(xi)
        p = np.empty_like(xi)
        cL = math.sqrt(g * pL / rhoL)
        cR = math.sqrt(g * pR / rhoR)
        for n, s in enumerate(xi):
            if s <= self.ustar:  # left of contact
                if self.left_shock:
                    if s <= self.SL:
                        r, uu, pp = rhoL, uL, pL
                    else:
                        r, uu, pp = self.rho_starL, self.ustar, self.pstar
                else:
                    if s <= self.SHL:
                        r, uu, pp = rhoL, uL, pL
                    elif s >= self.STL:
                        r, uu, pp = self.rho_starL, self.ustar, self.pstar
                    else:  # inside the left rarefaction fan
                        f = 2.0 / (g + 1) + (g - 1) / ((g + 1) * cL) * (uL - s)
                        r = rhoL * f ** (2.0 / (g - 1))
                        uu = 2.0 / (g + 1) * (cL + (g - 1) / 2.0 * uL + s)
                        pp = pL * f ** (2.0 * g / (g - 1))
            else:  # right of contact
                if self.right_shock:
                    if s >= self.SR:
                        r, uu, pp = rhoR, uR, pR
                    else:
                        r, uu, pp = self.rho_starR, self.ustar, self.pstar
                else:
                    if s >= self.SHR:
                        r, uu, pp = rhoR, uR, pR
                    elif s <= self.STR:
                        r, uu, pp = self.rho_starR, self.ustar, self.pstar
                    else:
                        f = 2.0 / (g + 1) - (g - 1) / ((g + 1) * cR) * (uR - s)
                        r = rhoR * f ** (2.0 / (g - 1))
                        uu = 2.0 / (g + 1) * (-cR + (g - 1) / 2.0 * uR + s)
                        pp = pR * f ** (2.0 * g / (g - 1))
            rho[n], u[n], p[n] = r, uu, pp
        e = p / ((g - 1.0) * rho)
        return rho, u, p, e


# --------------------------------------------------------------------------
# Sedov: energy constant of the self-similar spherical blast
# --------------------------------------------------------------------------
def sedov_alpha(gamma=1.4, eta_min=1e-6):
    """alpha such that R(t) = (E t^2 / (alpha rho0))^(1/5) for a spherical point
    blast in a uniform cold gas.

    Self-similar form behind the shock (eta = r/R, D = dR/dt = 2R/(5t)):
    u = D f(eta), rho = rho0 g(eta), p = rho0 D^2 h(eta). Substituting in the
    spherical Euler equations gives, with ' = d/deta,
        (f - eta) g' + g f' = -2 g f / eta               (mass)
        (f - eta) f' + h'/g = 3 f / 2                     (momentum)
        (f - eta) (h'/h - gamma g'/g) = 3                 (entropy along paths)
    with the strong-shock state f = 2/(gamma+1), g = (gamma+1)/(gamma-1),
    h = 2/(gamma+1) at eta = 1. The energy E = 4 pi rho0 D^2 R^3 I with
    I = int_0^1 (g f^2 / 2 + h / (gamma-1)) eta^2 deta, and D^2 R^3 =
    (4/25) R^5 / t^2, so alpha = 16 pi I / 25.
    """
    gm = gamma

    def rhs(eta, y):
        f, g, h = y
        a = f - eta
        # unknowns (f', g', h'): linear 3x3 system
        A = np.array([[g, a, 0.0],
                      [a, 0.0, 1.0 / g],
                      [0.0, -gm * a / g, a / h]])
        b = np.array([-2.0 * g * f / eta, 1.5 * f, 3.0])
        return np.linalg.solve(A, b)

    y0 = [2.0 / (gm + 1.0), (gm + 1.0) / (gm - 1.0), 2.0 / (gm + 1.0)]
    sol = solve_ivp(rhs, (1.0, eta_min), y0, method="DOP853", rtol=1e-12, atol=1e-14,
                    dense_output=True)
    if not sol.success:
        raise RuntimeError(sol.message)
    # energy integral by Gauss-Legendre on [eta_min, 1] (the integrand is smooth)
    xg, wg = np.polynomial.legendre.leggauss(400)
    etas = 0.5 * (1.0 - eta_min) * xg + 0.5 * (1.0 + eta_min)
    f, g, h = sol.sol(etas)
    integrand = (0.5 * g * f ** 2 + h / (gm - 1.0)) * etas ** 2
    I = 0.5 * (1.0 - eta_min) * np.sum(wg * integrand)
    return 16.0 * math.pi * I / 25.0


def sedov_radius(t, E=1.0, rho0=1.0, gamma=1.4):
    """Shock radius of the full-space point blast of energy E at time t."""
    return (E * t * t / (sedov_alpha(gamma) * rho0)) ** 0.2


# --------------------------------------------------------------------------
# Noh: closed-form implosion
# --------------------------------------------------------------------------
class NohExact:
    """Cold ideal gas (p = 0) of density rho0 moving at speed u0 toward the
    origin in `dims` dimensions (1 planar, 2 cylindrical, 3 spherical).

    Ahead of the shock the gas keeps its velocity -u0, so continuity with a
    converging cross-section r^(dims-1) gives rho = rho0 (1 + u0 t / r)^(dims-1)
    there. Behind it the gas is at rest. A strong shock in a cold gas
    compresses by (gamma+1)/(gamma-1); mass conservation in the shock frame
    (preshock speed u0 + D, postshock speed D) fixes the shock speed
    D = u0 (gamma-1)/2 and the postshock density
    rho0 ((gamma+1)/(gamma-1))^dims; the Hugoniot energy jump turns all the
    kinetic energy into internal energy, e = u0^2 / 2."""

    def __init__(self, gamma=5.0 / 3.0, u0=1.0, rho0=1.0, dims=3):
        if dims not in (1, 2, 3):
            raise ValueError("dims must be 1, 2 or 3")
        self.g, self.u0, self.rho0, self.dims = gamma, u0, rho0, dims
        self.D = u0 * (gamma - 1.0) / 2.0
        self.rho_post = rho0 * ((gamma + 1.0) / (gamma - 1.0)) ** dims
        self.e_post = 0.5 * u0 * u0

    def shock_radius(self, t):
        return self.D * t

    def sample(self, r, t):
        """(rho, u_r, p, e) at radii r (array, r > 0) and time t > 0."""
        r = np.asarray(r, dtype=np.float64)
        inside = r < self.D * t
        rho = np.where(inside, self.rho_post, self.rho0 * (1.0 + self.u0 * t / r) ** (self.dims - 1))
        u = np.where(inside, 0.0, -self.u0)
        e = np.where(inside, self.e_post, 0.0)
        p = (self.g - 1.0) * rho * e
        return rho, u, p, e
