"""Pins of the oracle's MRT collision (Eq. 2-5, Eq. 8) against textbook D2Q9 forms and
exact invariants."""
import numpy as np
import pytest

from oracle import lbm
from paper_1812_10375_amd import scenarios as S

E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(rho, u):
    eu = E @ u
    return W * rho * (1 + 3 * eu + 4.5 * eu**2 - 1.5 * (u @ u))


def textbook_guo(u, F):
    # velocity-space second-order forcing term w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)]
    return W * (3 * ((E - u) @ F) + 9 * (E @ u) * (E @ F))


def test_feq_is_the_textbook_equilibrium():
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.2, 7)
        u = rng.uniform(-0.1, 0.1, 2)
        assert lbm.feq(rho, *u) == pytest.approx(textbook_feq(rho, u), rel=1e-13, abs=1e-15)


def _rand_case(rng):
    rho = rng.uniform(0.3, 7)
    u = rng.uniform(-0.05, 0.05, 2)
    f = textbook_feq(rho, u) * (1 + rng.uniform(-0.05, 0.05, 9))
    F = rng.uniform(-0.05, 0.05, 2)
    Fm = rng.uniform(-0.05, 0.05, 2)
    return f, F, Fm


def test_collision_conserves_mass_and_adds_the_force():
    rng = np.random.default_rng(2)
    sc = S.base_params()
    for _ in range(50):
        f, F, Fm = _rand_case(rng)
        fs, ux, uy = lbm.collide_node(sc, f, F[0], F[1], Fm[0], Fm[1], 1.3)
        assert fs.sum() == pytest.approx(f.sum(), rel=1e-14)
        assert E.T @ fs == pytest.approx(E.T @ f + F, abs=1e-13)
        # Eq. 5: u = (sum e f + F/2) / rho
        assert (ux, uy) == pytest.approx(tuple((E.T @ f + F / 2) / f.sum()), abs=1e-15)


def test_equilibrium_is_a_fixed_point_without_force():
    rng = np.random.default_rng(3)
    sc = S.base_params()
    for _ in range(20):
        rho = rng.uniform(0.3, 7)
        u = rng.uniform(-0.05, 0.05, 2)
        f = textbook_feq(rho, u)
        fs, _, _ = lbm.collide_node(sc, f, 0, 0, 0, 0, 1.0)
        assert fs == pytest.approx(f, rel=1e-13, abs=1e-15)


def test_forcing_with_unit_rates_is_guo_bgk():
    # With every relaxation rate 1 and sigma = 0 the MRT step is BGK with tau = 1, and
    # Eq. 8's source must equal the textbook forcing: f* = f^eq(rho, u) + F_i / 2.
    # This fixes all nine entries of S, including the last one (u_x F_y + u_y F_x).
    rng = np.random.default_rng(4)
    sc = S.base_params(s_e=1.0, s_zeta=1.0, s_q=1.0, tau_l=1.0, tau_v=1.0, sigma=0.0)
    for _ in range(30):
        f, F, Fm = _rand_case(rng)
        fs, ux, uy = lbm.collide_node(sc, f, F[0], F[1], Fm[0], Fm[1], 1.0)
        u = np.array([ux, uy])
        expect = textbook_feq(f.sum(), u) + 0.5 * textbook_guo(u, F)
        assert fs == pytest.approx(expect, rel=1e-12, abs=1e-14)


def test_sigma_term_changes_only_e_and_zeta_moments():
    # The sigma term of Eq. 8 feeds the energy moments only: mass and momentum are
    # unchanged, and the difference lies in span{M row e, M row zeta}.
    rng = np.random.default_rng(5)
    sc1 = S.base_params()
    sc0 = S.base_params(sigma=0.0)
    e2 = (E**2).sum(1)
    re = -4 + 3 * e2
    rz = 4 - 10.5 * e2 + 4.5 * e2**2
    for _ in range(10):
        f, F, Fm = _rand_case(rng)
        a, _, _ = lbm.collide_node(sc1, f, F[0], F[1], Fm[0], Fm[1], 0.9)
        b, _, _ = lbm.collide_node(sc0, f, F[0], F[1], Fm[0], Fm[1], 0.9)
        d = a - b
        assert abs(d.sum()) < 1e-14 and np.abs(E.T @ d).max() < 1e-14
        coef, res, *_ = np.linalg.lstsq(np.c_[re, rz], d, rcond=None)
        assert np.abs(np.c_[re, rz] @ coef - d).max() < 1e-14
        assert np.abs(d).max() > 1e-8
