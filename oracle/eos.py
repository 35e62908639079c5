"""Peng-Robinson thermodynamics of the paper, in plain numpy/scipy (FP64).

TEST INFRASTRUCTURE (see the package docstring).

* Eq. 28 and Sec. 3.1: p(rho, T) with a = 3/49, b = 2/21, R = 1 and the standard
  Peng-Robinson alpha function phi(T) = [1 + kappa (1 - sqrt(T/Tc))]^2 (the printed
  form of phi is read this way; see ``maxwell`` and the tests).
* The coexistence densities the paper quotes in Sec. 3.1 are those of the Maxwell
  equal-area construction at T_s = 0.86 Tc.
* Eq. 14: latent heat h_lg = int_{v_l}^{v_v} T (dp/dT)_v dv.
"""
import math

import numpy as np
from scipy import integrate, optimize

A = 3.0 / 49.0
B = 2.0 / 21.0
R = 1.0


def Tc(a=A, b=B, R=R):
    """Sec. 3.1: a = 0.45724 R^2 Tc^2/pc, b = 0.0778 R Tc/pc  =>  Tc = (a/b)(0.0778/0.45724)/R."""
    return (a / b) * (0.0778 / 0.45724) / R


def pc(a=A, b=B, R=R):
    return 0.0778 * R * Tc(a, b, R) / b


def kappa(omega):
    """Sec. 3.1 (Eq. 28): kappa = 0.37464 + 1.54226 w - 0.26992 w^2."""
    return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega


def phi(T, omega, printed=False, a=A, b=B, R=R):
    """alpha function of Eq. 28.  printed=True evaluates the form exactly as printed."""
    t = T / Tc(a, b, R)
    k = kappa(omega)
    if printed:
        return (1.0 + k * np.sqrt(1.0 - t)) ** 2
    return (1.0 + k * (1.0 - np.sqrt(t))) ** 2


def dphi_dT(T, omega, a=A, b=B, R=R):
    tc = Tc(a, b, R)
    k = kappa(omega)
    s = 1.0 + k * (1.0 - np.sqrt(T / tc))
    return -k * s / np.sqrt(T * tc)


def pressure(rho, T, omega, printed=False, a=A, b=B, R=R):
    """Eq. 28."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho * R * T / (1.0 - b * rho) - a * phi(T, omega, printed, a, b, R) * rho**2 / (
        1.0 + 2.0 * b * rho - b * b * rho**2)


def dp_dT(rho, T, omega, a=A, b=B, R=R):
    """(dp/dT)_v of Eq. 28 (the factor in Eq. 13, 14 and 17)."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho * R / (1.0 - b * rho) - a * dphi_dT(T, omega, a, b, R) * rho**2 / (
        1.0 + 2.0 * b * rho - b * b * rho**2)


def psi(rho, T, omega, G=-1.0, printed=False):
    """Eq. 7 with c = 1, c_s^2 = 1/3: psi = sqrt(2 (p - rho/3) / G)."""
    return np.sqrt(2.0 * (pressure(rho, T, omega, printed) - np.asarray(rho) / 3.0) / G)


def _dp_drho(rho, T, omega, printed):
    h = 1e-6 * max(1.0, rho)
    return (pressure(rho + h, T, omega, printed) - pressure(rho - h, T, omega, printed)) / (2 * h)


def spinodals(T, omega, printed=False):
    """Densities where dp/drho = 0 (the van der Waals loop's extrema), found by scanning."""
    grid = np.linspace(1e-4, 1.0 / B - 1e-3, 20001)
    d = np.array([_dp_drho(r, T, omega, printed) for r in grid])
    idx = np.where(np.sign(d[:-1]) != np.sign(d[1:]))[0]
    roots = [optimize.brentq(lambda r: _dp_drho(r, T, omega, printed), grid[i], grid[i + 1])
             for i in idx]
    if len(roots) != 2:
        raise ValueError("no two-phase loop at T=%g" % T)
    return roots[0], roots[1]


def maxwell(T, omega, printed=False):
    """Maxwell equal-area construction: returns (rho_v, rho_l, p_sat).

    For a trial pressure p between the two spinodal pressures, the roots of
    p(rho) = p in the vapour and liquid branches are bracketed by the spinodals; p_sat
    is the pressure for which int_{v_l}^{v_v} p dv = p (v_v - v_l).
    """
    r1, r2 = spinodals(T, omega, printed)
    p_lo = max(float(pressure(r2, T, omega, printed)), 1e-14)
    p_hi = float(pressure(r1, T, omega, printed))
    rmax = 1.0 / B - 1e-9

    def roots(p0):
        f = lambda r: float(pressure(r, T, omega, printed)) - p0
        rv = optimize.brentq(f, 0.0, r1, xtol=1e-15)
        rl = optimize.brentq(f, r2, rmax, xtol=1e-15)
        return rv, rl

    def area(p0):
        rv, rl = roots(p0)
        vv, vl = 1.0 / rv, 1.0 / rl
        I, _ = integrate.quad(lambda v: float(pressure(1.0 / v, T, omega, printed)), vl, vv,
                              epsabs=0, epsrel=1e-13, limit=200)
        return I - p0 * (vv - vl)

    eps = 1e-12 * (p_hi - p_lo)
    psat = optimize.brentq(area, p_lo + eps, p_hi - eps, xtol=1e-16, rtol=1e-14)
    rv, rl = roots(psat)
    return rv, rl, psat


def latent_heat(T, omega):
    """Eq. 14: h_lg = int_{v_l}^{v_v} T (dp/dT)_v dv between the coexistence volumes."""
    rv, rl, _ = maxwell(T, omega)
    I, _ = integrate.quad(lambda v: T * float(dp_dT(1.0 / v, T, omega)), 1.0 / rl, 1.0 / rv,
                          epsabs=0, epsrel=1e-13, limit=200)
    return I


def latent_heat_clapeyron(T, omega, dT=None):
    """Independent route to the same number: h = T (v_v - v_l) dp_sat/dT (Clapeyron)."""
    if dT is None:
        dT = 1e-5 * T
    _, _, p_plus = maxwell(T + dT, omega)
    _, _, p_minus = maxwell(T - dT, omega)
    rv, rl, _ = maxwell(T, omega)
    return T * (1.0 / rv - 1.0 / rl) * (p_plus - p_minus) / (2.0 * dT)


def radicand_limit(T, omega, G=-1.0):
    """Smallest liquid-side density above which 2 (p - rho/3)/G <= 0 (psi undefined)."""
    f = lambda r: 2.0 * (float(pressure(r, T, omega)) - r / 3.0) / G
    grid = np.linspace(1.0, 1.0 / B - 1e-6, 4001)
    vals = np.array([f(r) for r in grid])
    i = np.where(vals <= 0)[0]
    if len(i) == 0:
        return math.inf
    i = i[0]
    return optimize.brentq(f, grid[i - 1], grid[i])
