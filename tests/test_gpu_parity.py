"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same
seeded inputs.  FP64 runs must agree to 1e-12 relative; FP32 runs to
max|drho|/rho_l <= 1e-4 over the pre-nucleation steps."""
import numpy as np
import pytest

from paper_1812_10375_amd import scenarios as S
from parity import errors, log, run_pair

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-4


def _check64(sc, steps, tol=TOL64):
    res, gpu, orc = run_pair(sc, steps)
    e = errors(res)
    log("[parity] errors %s" % {k: "%.2e" % v for k, v in e.items()})
    assert e["rho"] < tol and e["T"] < tol and e["u"] < 1e3 * tol, e
    og, oo = res["gpu_obs"], res["orc_obs"]
    assert og["step"] == oo["step"] == steps
    assert og["mass"] == pytest.approx(oo["mass"], rel=tol)
    for k in ("dE_cum", "Q_bottom_cum", "Q_top_cum", "Q_surface_cum", "energy"):
        assert og[k] == pytest.approx(oo[k], rel=1e-10, abs=1e-12 * max(1.0, abs(oo["Q_bottom_cum"]))), k
    # the per-step fluxes and their running mean and variance (time averages of Sec. 4.4)
    qs = max(abs(oo["q_bottom_mean"]), abs(oo["q_bottom"]), 1e-300)
    for k in ("q_bottom", "q_surface", "q_bottom_mean"):
        assert og[k] == pytest.approx(oo[k], rel=1e-10, abs=1e-12 * qs), k
    assert og["q_bottom_var"] == pytest.approx(oo["q_bottom_var"], rel=1e-8, abs=1e-12 * qs * qs)
    # the library reports the rho_ave of Eq. 9 that the next step uses (the mass after
    # this step over the fluid nodes); the oracle's record holds the one this step used
    assert og["rho_ave"] == pytest.approx(oo["mass"] / (sc["nx"] * sc["ny"]), rel=tol)
    assert og["max_speed"] == pytest.approx(oo["max_speed"], rel=1e-9, abs=1e-15)
    return res, e


def test_fp64_interface_conduction_exact_energy():
    # 8 x 256, walls at 0.87 Tc and 0.85 Tc, stagnant, no latent heat (Sec. 3.2 setting)
    sc = S.interface_conduction(steps=1000)
    res, e = _check64(sc, 1000)
    og = res["gpu_obs"]
    # the GPU conserves energy exactly too: stored change == heat through the walls
    assert og["dE_cum"] == pytest.approx(og["Q_bottom_cum"] + og["Q_top_cum"], rel=1e-12)


def test_fp64_interface_conduction_full_physics():
    sc = S.interface_conduction(exact_energy=False, steps=1000)
    _check64(sc, 1000)


def test_fp64_ragged_pool_boiling():
    # ragged in x (100 = 64 + 36) and in both T and fluid rows; heater, sites, gravity,
    # convective outlet
    sc = S.pool_boiling(nx=100, ny=70, heater_rows=5, n_sites=2, min_spacing=20, seed=5,
                        precision="f64")
    _check64(sc, 300)


def test_fp64_tall_domain_with_interior_tiles():
    # tall enough that some energy tiles have a halo without heater or ghost rows
    sc = S.pool_boiling(nx=40, ny=200, heater_rows=5, n_sites=1, min_spacing=8, seed=9,
                        precision="f64")
    _check64(sc, 300)


def test_fp64_film_constant_pressure_top():
    sc = S.film_evaporation(nx=70, ny=50, film=12, superheat=0.05, seed=7, precision="f64")
    _check64(sc, 300)


def test_fp64_film_evaporation_1000_steps():
    # the 256 x 256 film-evaporation workload (Dirichlet wall, 40-row film, seeded
    # perturbation, constant-pressure top) in FP64 over 1000 steps
    sc = S.film_evaporation(precision="f64")
    _check64(sc, 1000)


def test_fp64_pool_boiling_cropped_1000_steps():
    # the pool-boiling workload cropped to 256 x 256 (25-row heater, sites, gravity,
    # convective outlet, 70% liquid) in FP64 over 1000 steps
    sc = S.pool_boiling(nx=256, ny=256, n_sites=2, min_spacing=64, seed=3, precision="f64")
    _check64(sc, 1000)


@pytest.mark.parametrize("nx,ny,nh", [(1, 12, 0), (3, 2, 2), (65, 17, 1)])
def test_fp64_degenerate_shapes(nx, ny, nh):
    sc = S.pool_boiling(nx=nx, ny=ny, heater_rows=nh, n_sites=0, seed=1, precision="f64")
    _check64(sc, 50)


def test_fp64_energy_substeps_and_flux_bottom():
    sc = S.film_evaporation(nx=40, ny=30, film=10, seed=3, precision="f64")
    sc["n_sub"] = 3
    sc["bottom_tbc"] = "flux"
    sc["q_bottom"] = 2e-4
    sc["heater_rows"] = 4
    sc["T0"] = np.full((34, 40), S.T_SAT)
    _check64(sc, 100)


def test_fp64_isotropic_comparison_scheme():
    sc = S.interface_conduction(nx=8, ny=64, steps=200)
    sc["flags"] = ("freeze_eos_T", "no_advection", "no_latent", "diff_isotropic")
    _check64(sc, 200)


def test_zero_steps_leave_the_state():
    from paper_1812_10375_amd.lbm import Lattice
    sc = S.film_evaporation(nx=33, ny=20, film=6, precision="f64")
    gpu = Lattice(sc)
    gpu.step(0)
    ob = gpu.observe()
    assert ob["step"] == 0
    assert gpu.read("T") == pytest.approx(sc["T0"], abs=0)
    assert ob["mass"] == pytest.approx(sc["rho0"].sum(), rel=1e-14)


def _check32(sc, steps):
    res, gpu, orc = run_pair(sc, steps)
    e = errors(res)
    log("[parity] errors %s" % {k: "%.2e" % v for k, v in e.items()})
    assert e["rho"] < TOL32, e
    assert e["T"] < TOL32, e
    og, oo = res["gpu_obs"], res["orc_obs"]
    assert og["mass"] == pytest.approx(oo["mass"], rel=1e-6)
    return res, e


def _trajectory32(sc, steps=1000, every=100):
    """FP32 path against the oracle every `every` steps: max|drho|/rho_l (bound TOL32 at
    every checkpoint) and max|dT| over the wall superheat (reported)."""
    from oracle.lbm import OracleSim
    from paper_1812_10375_amd.lbm import Lattice
    log("[parity] %s nx=%d ny=%d nh=%d FP32 trajectory over %d steps" % (
        sc.get("name", "?"), sc["nx"], sc["ny"], sc["heater_rows"], steps))
    gpu, orc = Lattice(sc), OracleSim(sc)
    dTw = abs(sc["T_bottom"] - S.T_SAT)
    worst = 0.0
    for n in range(every, steps + 1, every):
        gpu.step(every)
        assert orc.step(every) == 0, "oracle flagged an error"
        gpu.observe()
        er = np.abs(gpu.read("rho") - orc.field("rho")).max() / S.RHO_L
        eT = np.abs(gpu.read("T") - orc.field("T")).max() / dTw
        log("[parity]   step %4d  max|drho|/rho_l %.2e  max|dT|/dT_wall %.2e" % (n, er, eT))
        assert er <= TOL32, (n, er)
        worst = max(worst, er)
    return worst


def test_fp32_film_evaporation_1000_steps():
    sc = S.film_evaporation(steps=1000)     # 256 x 256, the film-evaporation workload
    _check32(sc, 1000)


def test_fp32_pool_boiling_cropped_1000_steps():
    sc = S.pool_boiling(nx=256, ny=256, n_sites=2, min_spacing=64, seed=3)
    _check32(sc, 1000)


def test_fp32_error_trajectory_film_evaporation():
    _trajectory32(S.film_evaporation(steps=1000))


def test_fp32_error_trajectory_pool_boiling_cropped():
    _trajectory32(S.pool_boiling(nx=256, ny=256, n_sites=2, min_spacing=64, seed=3))


def test_fp32_pool_boiling_full_size_first_steps():
    # the 1024 x 1024 + 25-row heater workload in the launch configuration the
    # benchmark times, against the oracle over its first steps
    sc = S.pool_boiling()
    _check32(sc, 20)


def test_fp32_error_trajectory_pool_boiling_full_size():
    # the full 1024 x 1024 + 25 workload (8 sites, 70% pool, convective outlet; the fused
    # step at this size) against the oracle every 100 steps over the first 1000 steps
    worst = _trajectory32(S.pool_boiling())
    log("[parity] 1024 x 1024 + 25 worst max|drho|/rho_l over 1000 steps %.2e" % worst)


def test_fp32_pool_boiling_4096_first_steps():
    # the 4096 x 4096 + 25 workload the benchmark times for HBM-resident rates: many
    # rounds of energy workgroups and 67 MB field planes
    sc = S.pool_boiling(nx=4096, ny=4096)
    _check32(sc, 3)


def _check32_heat(sc, steps, rel=1e-3):
    res, e = _check32(sc, steps)
    og, oo = res["gpu_obs"], res["orc_obs"]
    scale = max(abs(oo["Q_bottom_cum"]), abs(oo["Q_top_cum"]), 1e-30)
    for k in ("Q_bottom_cum", "Q_top_cum", "Q_surface_cum", "dE_cum"):
        assert abs(og[k] - oo[k]) <= rel * scale, (k, og[k], oo[k])
    return res, e


def test_fp32_interface_conduction_walls():
    # Dirichlet walls below and above (Sec. 3.2 setting), FP32 fields
    sc = S.interface_conduction(exact_energy=False, steps=1000)
    sc["precision"] = "f32"
    _check32_heat(sc, 1000)


def test_fp32_tall_domain_with_interior_tiles():
    sc = S.pool_boiling(nx=40, ny=200, heater_rows=5, n_sites=1, min_spacing=8, seed=9)
    _check32_heat(sc, 300)


@pytest.mark.parametrize("nx,ny,nh,rows", [(128, 256, 25, 44), (96, 300, 12, 40)])
def test_fp32_shaped_edge_tile_rows(nx, ny, nh, rows):
    # with these heights the FP32 energy grid shortens its first and last tile rows
    # (first 31 or 30 rows, interior 44 or 42, last 30), so tiles of three heights and
    # both code paths meet at the tile-row seams
    sc = S.pool_boiling(nx=nx, ny=ny, heater_rows=nh, n_sites=2, min_spacing=32, seed=5)
    sc["tile_rows"] = rows
    _check32_heat(sc, 1000)


def test_fp32_energy_substeps_and_flux_bottom():
    sc = S.film_evaporation(nx=40, ny=30, film=10, seed=3, precision="f32")
    sc["n_sub"] = 3
    sc["bottom_tbc"] = "flux"
    sc["q_bottom"] = 2e-4
    sc["heater_rows"] = 4
    sc["T0"] = np.full((34, 40), S.T_SAT)
    _check32_heat(sc, 100)


@pytest.mark.parametrize("nx,ny,nh", [(1, 12, 0), (3, 2, 2), (65, 17, 1), (130, 90, 25)])
def test_fp32_degenerate_and_ragged_shapes(nx, ny, nh):
    sc = S.pool_boiling(nx=nx, ny=ny, heater_rows=nh, n_sites=0, seed=1, precision="f32")
    _check32(sc, 50)


def test_fp32_isotropic_comparison_scheme():
    # the comparison scheme of Eq. 20-21 in FP32 (the LDS energy kernel), across a flat
    # interface between Dirichlet walls
    sc = S.interface_conduction(nx=8, ny=64, steps=200)
    sc["flags"] = ("freeze_eos_T", "no_advection", "no_latent", "diff_isotropic")
    sc["precision"] = "f32"
    _check32_heat(sc, 200)


@pytest.mark.parametrize("isotropic", [False, True])
def test_fp32_flux_driven_film_with_a_conductive_wall(isotropic):
    # the Sec. 3.3 film at its paper size in FP32: 20-row wall at three times the
    # liquid's conductivity, heat flux through the bottom, constant-pressure top, five
    # energy sub-steps per LB step (Eq. 27), both diffusion schemes.  The heat through
    # the bottom is q per unit length and step in both.  The stored-energy change sums
    # rho c_v dT over the run; with the wall's heat capacity large against the heat let
    # in, its FP32 difference is bounded by the fields' instead: about sum(rho c_v) max|dT|.
    sc = S.film_evaporation_flux(3.0, 2e-4, precision="f32", isotropic=isotropic)
    steps = 300
    res, e = _check32(sc, steps)
    og, oo = res["gpu_obs"], res["orc_obs"]
    assert og["Q_bottom_cum"] == pytest.approx(2e-4 * sc["nx"] * steps, rel=1e-6)
    assert og["Q_bottom_cum"] == pytest.approx(oo["Q_bottom_cum"], rel=1e-6)
    cap = sc["rho_w"] * sc["cv_w"] * sc["heater_rows"] * sc["nx"] + (res["rho"][1] * sc["cv"]).sum()
    dT = np.abs(res["T"][0] - res["T"][1]).max()
    log("[parity] dE_cum GPU %.6f oracle %.6f; bound %.6f" % (og["dE_cum"], oo["dE_cum"], 2 * cap * dT))
    # (twice the bound: rho of each step, not only the last, weighs the increments)
    assert abs(og["dE_cum"] - oo["dE_cum"]) <= 2 * cap * dT
