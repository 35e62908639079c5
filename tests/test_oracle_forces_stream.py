"""Pins of the oracle's forces (Eq. 6, Eq. 9, Eq. 10) and streaming/boundaries (Eq. 1)."""
import numpy as np
import pytest

from oracle import lbm
from paper_1812_10375_amd import scenarios as S


def _sim(nx, ny, **kw):
    sc = S.base_params(nx=nx, ny=ny, **kw)
    sc.setdefault("rho0", np.full((ny, nx), S.RHO_L))
    sc.setdefault("T0", np.full((sc["heater_rows"] + ny, nx), S.T_SAT))
    return lbm.OracleSim(sc), sc


def test_interaction_force_is_minus_G_psi_grad_psi_on_linear_psi():
    # sum_i w_i e_i e_i = I for w = (1/3, 1/12), so on a linear psi the stencil of Eq. 6
    # returns -G psi grad psi exactly (away from walls).
    o, sc = _sim(6, 16, g=0.0)
    y = np.arange(16)[:, None] * np.ones((1, 6))
    a, b = 1.1, 0.037
    o.set_field("psi", a + b * y)
    o.forces()
    fmx, fmy = o.field("Fmx"), o.field("Fmy")
    G = sc["G"]
    assert np.abs(fmx).max() < 1e-15
    assert fmy[1:-1] == pytest.approx((-G * (a + b * y) * b)[1:-1], rel=1e-13)


def test_uniform_psi_feels_no_force_next_to_neutral_walls():
    o, _ = _sim(5, 7, g=0.0, Gw0=0.0, Gw_top=0.0)
    o.set_field("psi", np.full((7, 5), 1.7))
    o.forces()
    assert np.abs(o.field("Fx")).max() < 1e-15
    assert np.abs(o.field("Fy")).max() < 1e-15


def test_adhesion_closed_form():
    # Eq. 10 with omega = w/3: the three solid neighbours below a bottom-row node weigh
    # 1/9 + 2/36 = 1/6, so F_ads,y = -G_w psi^2 / 6 (and +G_w,top psi^2 / 6 under a top wall).
    o, _ = _sim(5, 7, g=0.0, Gw0=0.3, Gw_top=0.12)
    psi = 1.7
    o.set_field("psi", np.full((7, 5), psi))
    o.forces()
    fy = o.field("Fy")
    assert fy[0] == pytest.approx(np.full(5, -0.3 * psi**2 / 6), rel=1e-14)
    assert fy[-1] == pytest.approx(np.full(5, 0.12 * psi**2 / 6), rel=1e-14)
    assert np.abs(fy[1:-1]).max() < 1e-15
    assert np.abs(o.field("Fx")).max() < 1e-15


def test_adhesion_x_component_over_a_site():
    # Over a nucleation site G_w varies along the wall; the diagonal solid neighbours
    # then give F_ads,x = psi^2 (G_w(x+1) - G_w(x-1)) / 36.
    nx = 24
    o, _ = _sim(nx, 6, g=0.0, Gw0=0.3, sites=np.array([[10.0, 6.0, -0.6]]))
    psi = 2.0
    o.set_field("psi", np.full((6, nx), psi))
    o.forces()
    gw = o.field("Gw")
    fx = o.field("Fx")[0]
    expect = psi**2 * (np.roll(gw, -1) - np.roll(gw, 1)) / 36.0
    assert fx == pytest.approx(expect, abs=1e-14)
    assert np.abs(fx).max() > 1e-3


def test_site_profile_shape():
    nx = 40
    o, _ = _sim(nx, 4, Gw0=0.3, sites=np.array([[20.0, 10.0, -0.3], [1.0, 4.0, 0.0]]))
    gw = o.field("Gw")
    inside = np.abs(np.arange(nx) + 0.5 - 20.0) < 5.0
    assert np.all(gw[~inside & (np.arange(nx) > 5) & (np.arange(nx) < 35)] == 0.3)
    assert np.all(gw[inside] < 0.3) and gw.min() > -0.3
    assert gw[15:25] == pytest.approx(gw[15:25][::-1])           # symmetric about x_c
    assert np.all(np.diff(gw[15:20]) < 0)                         # linear drop to the centre
    assert gw[-1] < 0.3 and gw[0] < 0.3 and gw[2] < 0.3           # a site wraps round x = 0


def test_buoyancy_uses_the_domain_mean_density():
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.4, 6.4, (9, 7))
    o, sc = _sim(7, 9, g=3e-5, rho0=rho)
    o.set_field("psi", np.full((9, 7), 1.0))
    o.set_field("rho", rho)
    o.forces()
    fy = o.field("Fy")
    fy[0] += 0.0  # neutral walls contribute nothing here (Gw = 0, uniform psi)
    assert fy == pytest.approx(-(rho - rho.mean()) * 3e-5, abs=1e-18)
    assert abs(fy.sum()) < 1e-15


def test_mirror_in_x_flips_the_x_force():
    rng = np.random.default_rng(6)
    psi = rng.uniform(0.4, 2.1, (10, 8))
    sites = np.array([[3.0, 4.0, -0.3]])
    o1, _ = _sim(8, 10, g=0.0, Gw0=0.3, sites=sites)
    o2, _ = _sim(8, 10, g=0.0, Gw0=0.3, sites=np.array([[8 - 3.0, 4.0, -0.3]]))
    o1.set_field("psi", psi)
    o2.set_field("psi", psi[:, ::-1])
    o1.forces()
    o2.forces()
    assert o2.field("Fx")[:, ::-1] == pytest.approx(-o1.field("Fx"), abs=1e-14)
    assert o2.field("Fy")[:, ::-1] == pytest.approx(o1.field("Fy"), abs=1e-14)


def test_translation_in_x_commutes_with_a_step():
    sc = S.film_evaporation(nx=12, ny=16, film=6, steps=5)
    sc["sites"] = np.array([[4.0, 4.0, 0.0]])
    a = lbm.OracleSim(sc)
    sc2 = dict(sc)
    sc2["rho0"] = np.roll(sc["rho0"], 5, axis=1)
    sc2["T0"] = np.roll(sc["T0"], 5, axis=1)
    sc2["sites"] = np.array([[9.0, 4.0, 0.0]])
    b = lbm.OracleSim(sc2)
    a.step(20)
    b.step(20)
    assert np.roll(a.field("rho"), 5, axis=1) == pytest.approx(b.field("rho"), rel=1e-12)
    assert np.roll(a.field("T"), 5, axis=1) == pytest.approx(b.field("T"), rel=1e-12)


def test_uniform_fluid_at_rest_stays_at_rest():
    o, _ = _sim(6, 5, g=3e-5, Gw0=0.0)
    f0 = o.field("f")
    o.step(50)
    assert o.field("f") == pytest.approx(f0, rel=1e-13)
    assert np.abs(o.field("ux")).max() < 1e-14 and np.abs(o.field("uy")).max() < 1e-14


def test_closed_box_conserves_mass():
    sc = S.interface_conduction(nx=4, ny=64)
    sc["rho0"] = sc["rho0"] + np.random.default_rng(1).uniform(-0.01, 0.01, sc["rho0"].shape)
    o = lbm.OracleSim(sc)
    m0 = o.observe()["mass"]
    o.step(500)
    assert o.observe()["mass"] == pytest.approx(m0, rel=1e-13)
