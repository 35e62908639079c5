"""Validation of the oracle as a whole against what the paper and physics fix: phase
coexistence (Sec. 3.1), the wall's contact angle (Sec. 4.2), the Laplace law, and the
phase viscosities (Sec. 3.1).  These runs pin readings of the paper that no single
formula settles; each takes seconds to tens of seconds on the CPU."""
import numpy as np
import pytest

from oracle import eos, lbm
from paper_1812_10375_amd import scenarios as S

ISO = ("freeze_eos_T", "no_advection", "no_latent")


def _flat_interface(flags, steps=20000):
    sc = S.interface_conduction(nx=4, ny=256)
    sc["flags"] = flags
    sc["T_bottom"] = sc["T_top"] = S.T_SAT
    o = lbm.OracleSim(sc)
    o.step(steps)
    rho = o.field("rho")
    return rho[40:90].mean(), rho[170:220].mean()


@pytest.mark.slow
def test_coexistence_matches_maxwell_with_the_12_sigma_reading():
    # Sec. 3.1 chooses sigma = 0.107 for thermodynamic consistency; the relaxed bulk
    # densities then match the Maxwell construction only if Eq. 8's sigma terms carry
    # the factor 12 of the forcing scheme it adopts.
    rv, rl, _ = eos.maxwell(S.T_SAT, S.OMEGA)
    liq, vap = _flat_interface(ISO)
    assert liq == pytest.approx(rl, rel=0.005)
    assert vap == pytest.approx(rv, rel=0.03)
    liq0, vap0 = _flat_interface(ISO + ("sigma_plain",))
    assert abs(vap0 - rv) / rv > 0.3


def _contact_angle(rho, nx, ny):
    mid = 0.5 * (S.RHO_L + S.RHO_V)
    pts = []
    for y in range(3, ny):
        row = rho[y]
        idx = np.where(row > mid)[0]
        if len(idx) == 0:
            break
        i0, i1 = idx[0], idx[-1]
        assert 0 < i0 and i1 < nx - 1, "drop spread over the whole wall"
        xl = i0 - 1 + (mid - row[i0 - 1]) / (row[i0] - row[i0 - 1])
        xr = i1 + (row[i1] - mid) / (row[i1] - row[i1 + 1])
        pts += [(xl + 0.5, y + 0.5), (xr + 0.5, y + 0.5)]
    P = np.array(pts)
    A = np.c_[2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))]
    cx, cy, c = np.linalg.lstsq(A, (P**2).sum(1), rcond=None)[0]
    r = np.sqrt(c + cx * cx + cy * cy)
    # the half-way bounce-back wall lies at y = 0 in node-centre coordinates
    return np.degrees(np.arccos(np.clip(-cy / r, -1, 1)))


@pytest.mark.slow
def test_contact_angle_at_Gw_0p3(paper):
    # Sec. 4.2: G_w = 0.3 gives a contact angle of about 35 degrees.  This fixes the
    # wall readings of Eq. 6 (a solid neighbour carries psi(x)) and Eq. 10 (weights
    # w/3 = 1/9, 1/36); other readings give complete wetting or > 60 degrees.
    nx, ny = 260, 60
    sc = S.sessile_drop(nx, ny, 22, 0.3)
    o = lbm.OracleSim(sc)
    o.step(15000)
    theta = _contact_angle(o.field("rho"), nx, ny)
    pv = paper["contact_angle_deg_Gw_0p3"]
    assert theta == pytest.approx(pv["value"], abs=pv["abs_tol_deg"])


@pytest.mark.slow
def test_laplace_law_for_static_bubbles():
    n = 80
    pts = []
    for R in (10, 16, 22):
        sc = S.static_droplet(n, n, R, bubble=True)
        o = lbm.OracleSim(sc)
        o.step(8000)
        rho, psi = o.field("rho"), o.field("psi")
        p = rho / 3 + sc["G"] * psi**2 / 2          # Eq. 7
        dp = p[n // 2 - 1:n // 2 + 1, n // 2 - 1:n // 2 + 1].mean() - p[5:10].mean()
        reff = np.sqrt((rho < 0.5 * (S.RHO_L + S.RHO_V)).sum() / np.pi)
        pts.append((reff, dp))
    a = np.array(pts)
    A = np.c_[1 / a[:, 0], np.ones(len(a))]
    coef = np.linalg.lstsq(A, a[:, 1], rcond=None)[0]
    pred = A @ coef
    r2 = 1 - ((a[:, 1] - pred) ** 2).sum() / ((a[:, 1] - a[:, 1].mean()) ** 2).sum()
    assert np.all(a[:, 1] > 0) and np.all(np.diff(a[:, 1]) < 0)
    assert r2 > 0.99
    assert 0.05 < coef[0] < 0.3      # surface tension, lattice units


@pytest.mark.parametrize("rho,nu_key", [(S.RHO_L, "nu_l"), (S.RHO_V, "nu_v")])
def test_shear_wave_decay_gives_the_phase_viscosity(paper, rho, nu_key):
    # Sec. 3.1: nu_l = 0.1, nu_v = 0.5/3 through nu = (tau - 1/2)/3.  A shear wave
    # u_x = U sin(2 pi m x / n)... here along y between the no-slip walls: the first
    # mode sin(pi (y + 1/2) / ny) decays as exp(-nu (pi/ny)^2 t).
    nx, ny = 2, 48
    y = np.arange(ny) + 0.5
    U = 1e-4
    ux = U * np.sin(np.pi * y / ny)
    sc = S.base_params(nx=nx, ny=ny, flags=ISO)
    sc["rho0"] = np.full((ny, nx), rho)
    sc["T0"] = np.full((ny, nx), S.T_SAT)
    o = lbm.OracleSim(sc)
    f = np.stack([np.stack([lbm.feq(rho, ux[j], 0.0) for _ in range(nx)]) for j in range(ny)])
    o.set_field("f", np.transpose(f, (2, 0, 1)))
    amps = []
    for _ in range(3):
        o.step(1000)
        u = o.field("ux")[:, 0]
        amps.append((u * np.sin(np.pi * y / ny)).sum() / (np.sin(np.pi * y / ny) ** 2).sum())
    rate = np.log(amps[1] / amps[2]) / 1000.0
    nu = rate / (np.pi / ny) ** 2
    assert nu == pytest.approx(paper[nu_key]["value"], rel=0.02)


@pytest.mark.parametrize("frac", [0.1, 0.75])
def test_shear_wave_decay_follows_the_linear_relaxation_time(frac):
    # Between the phases tau varies linearly in rho (the reading of Sec. 3.1 taken here).
    # A uniform fluid at a metastable density (vapour side, liquid side: outside the
    # spinodal, so it stays uniform) decays a shear wave at nu = (tau(rho) - 1/2)/3.
    nx, ny = 2, 48
    rho = S.RHO_V + frac * (S.RHO_L - S.RHO_V)
    y = np.arange(ny) + 0.5
    ux = 1e-4 * np.sin(np.pi * y / ny)
    sc = S.base_params(nx=nx, ny=ny, flags=ISO)
    sc["rho0"] = np.full((ny, nx), rho)
    sc["T0"] = np.full((ny, nx), S.T_SAT)
    o = lbm.OracleSim(sc)
    f = np.stack([np.stack([lbm.feq(rho, ux[j], 0.0) for _ in range(nx)]) for j in range(ny)])
    o.set_field("f", np.transpose(f, (2, 0, 1)))
    amps = []
    for _ in range(3):
        o.step(1000)
        u = o.field("ux")[:, 0]
        amps.append((u * np.sin(np.pi * y / ny)).sum() / (np.sin(np.pi * y / ny) ** 2).sum())
    r = o.field("rho")
    assert r.max() - r.min() < 1e-4 * rho
    nu = np.log(amps[1] / amps[2]) / 1000.0 / (np.pi / ny) ** 2
    tau = sc["tau_v"] + (sc["tau_l"] - sc["tau_v"]) * frac
    assert nu == pytest.approx((tau - 0.5) / 3.0, rel=5e-3)
