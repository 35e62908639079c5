"""Pins of the oracle's thermodynamics (Eq. 7, Eq. 14, Eq. 28, Sec. 3.1, Sec. 3.3).

Each test checks the oracle against something other than itself: the critical-point
conditions of the Peng-Robinson form, the numbers the paper prints, the Clapeyron
equation, and finite differences.
"""
import numpy as np
import pytest

from oracle import eos, lbm
from paper_1812_10375_amd import scenarios as S


def test_tc_is_the_critical_point():
    # At Tc (phi = 1) the isotherm has a horizontal inflection: min dp/drho = 0;
    # slightly below Tc it has a van der Waals loop, slightly above it is monotone.
    tc = eos.Tc()
    rho = np.linspace(0.5, 6.0, 200001)

    def min_slope(T):
        p = eos.pressure(rho, T, S.OMEGA)
        return np.min(np.diff(p) / np.diff(rho))

    # (0.0778 and 0.45724 are rounded Peng-Robinson constants, so the inflection sits
    # within ~2e-5 of Tc rather than exactly on it)
    assert abs(min_slope(tc)) < 2e-5
    assert min_slope(0.999 * tc) < 0 < min_slope(1.001 * tc)
    # and the critical pressure is the pc of the a, b definitions (Sec. 3.1)
    i = np.argmin(np.abs(np.diff(eos.pressure(rho, tc, S.OMEGA))))
    assert eos.pressure(rho[i], tc, S.OMEGA) == pytest.approx(eos.pc(), rel=1e-3)


def test_scenario_constants_are_the_eos_values():
    rv, rl, _ = eos.maxwell(S.T_SAT, S.OMEGA)
    assert S.TC == pytest.approx(eos.Tc(), rel=1e-15)
    assert S.RHO_L == pytest.approx(rl, rel=1e-10)
    assert S.RHO_V == pytest.approx(rv, rel=1e-10)


def test_coexistence_densities_match_paper(paper):
    rv, rl, psat = eos.maxwell(S.T_SAT, S.OMEGA)
    assert round(rl, paper["coexistence_rho_l"]["digits"]) == paper["coexistence_rho_l"]["value"]
    assert round(rv, paper["coexistence_rho_v"]["digits"]) == paper["coexistence_rho_v"]["value"]
    # equal pressure on both branches
    assert eos.pressure(rl, S.T_SAT, S.OMEGA) == pytest.approx(psat, rel=1e-9)
    assert eos.pressure(rv, S.T_SAT, S.OMEGA) == pytest.approx(psat, rel=1e-9)


def test_printed_alpha_function_contradicts_paper(paper):
    # Eq. 28 as printed, phi = [1 + kappa sqrt(1 - T/Tc)]^2, cannot give rho_l ~ 6.5,
    # rho_v ~ 0.38: the oracle reads phi as the standard Peng-Robinson form.
    rv, rl, _ = eos.maxwell(S.T_SAT, S.OMEGA, printed=True)
    assert abs(rl - paper["coexistence_rho_l"]["value"]) > 1.0
    assert abs(rv - paper["coexistence_rho_v"]["value"]) > 0.3


def test_latent_heat_eq14_equals_clapeyron_and_paper(paper):
    h14 = eos.latent_heat(S.T_SAT, S.OMEGA)
    hcl = eos.latent_heat_clapeyron(S.T_SAT, S.OMEGA)
    assert h14 == pytest.approx(hcl, rel=1e-6)
    pv = paper["latent_heat_0p86Tc"]
    assert h14 == pytest.approx(pv["value"], rel=pv["rel_tol"])


def test_c_oracle_eos_matches_python():
    sc = S.base_params()
    for rho in np.linspace(0.1, 8.0, 23):
        for tr in (0.8, 0.86, 0.9, 0.97):
            T = tr * S.TC
            assert lbm.eos_p(sc, rho, T) == pytest.approx(float(eos.pressure(rho, T, S.OMEGA)), rel=1e-13, abs=1e-15)
            assert lbm.dpdT(sc, rho, T) == pytest.approx(float(eos.dp_dT(rho, T, S.OMEGA)), rel=1e-13)
            ps = lbm.psi(sc, rho, T)
            if np.isfinite(ps):
                # Eq. 7 round trip: p = rho/3 + G psi^2 / 2
                assert rho / 3.0 + sc["G"] * ps * ps / 2.0 == pytest.approx(lbm.eos_p(sc, rho, T), rel=1e-12, abs=1e-14)
    assert lbm.Tc(sc) == pytest.approx(eos.Tc(), rel=1e-15)


def test_dpdT_is_the_temperature_derivative():
    for rho in (0.38, 2.0, 4.0, 6.5):
        for T in (0.8 * S.TC, S.T_SAT, 0.95 * S.TC):
            h = 1e-6 * T
            fd = (eos.pressure(rho, T + h, S.OMEGA) - eos.pressure(rho, T - h, S.OMEGA)) / (2 * h)
            assert float(eos.dp_dT(rho, T, S.OMEGA)) == pytest.approx(float(fd), rel=1e-7)


def test_psi_defined_up_to_radicand_limit():
    lim = eos.radicand_limit(S.T_SAT, S.OMEGA)
    sc = S.base_params()
    assert 8.9 < lim < 9.05
    assert np.isfinite(lbm.psi(sc, lim - 1e-3, S.T_SAT))
    assert np.isnan(lbm.psi(sc, lim + 1e-3, S.T_SAT))
