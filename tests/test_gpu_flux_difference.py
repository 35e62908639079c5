"""Sec. 3.2 on the GPU: heat conduction across a flat liquid-vapour interface between
walls held at T_h = 1 and T_l = 0 (EOS temperature frozen, no advection, no latent
heat).  At steady state the heat entering through the hot wall leaves through the cold
one: the relative flux difference is below 1e-10 with the finite-volume faces of
Eq. 22-26 and about 0.18 with the isotropic central scheme of Eq. 20-21."""
import numpy as np
import pytest

from paper_1812_10375_amd import scenarios as S
from parity import log

pytestmark = pytest.mark.gpu

NY = 40


def _relaxed_density():
    from paper_1812_10375_amd.lbm import Lattice
    sc = S.interface_conduction(nx=2, ny=NY)
    sc["T_bottom"] = sc["T_top"] = S.T_SAT
    lat = Lattice(sc)
    lat.step(20000)
    lat.observe()
    return lat.read("rho")


@pytest.fixture(scope="module")
def relaxed():
    return _relaxed_density()


def _flux_difference(rho, isotropic):
    from paper_1812_10375_amd.lbm import Lattice
    sc = S.interface_conduction(nx=2, ny=NY)
    if isotropic:
        sc["flags"] = tuple(sc["flags"]) + ("diff_isotropic",)
    sc["T_bottom"], sc["T_top"] = 1.0, 0.0
    sc["rho0"] = rho
    sc["T0"] = np.full((NY, 2), 0.5)
    lat = Lattice(sc)
    lat.step(int(40 * NY * NY / (np.pi ** 2 * sc["k"])))
    a = lat.observe()
    lat.step(1)
    b = lat.observe()
    qh = b["Q_bottom_cum"] - a["Q_bottom_cum"]
    ql = -(b["Q_top_cum"] - a["Q_top_cum"])
    return 2 * abs(qh - ql) / (qh + ql)


def test_flux_difference_finite_volume(relaxed):
    d = _flux_difference(relaxed, isotropic=False)
    log("[flux] FV relative flux difference %.3e" % d)
    assert d < 1e-10


def test_flux_difference_isotropic(relaxed):
    d = _flux_difference(relaxed, isotropic=True)
    log("[flux] isotropic relative flux difference %.4f" % d)
    assert d == pytest.approx(0.18, abs=0.015)
