"""Once pool boiling is under way, FP32 runs leave the FP64 trajectory pointwise; the
comparable result is then the time-averaged wall heat flux (Sec. 4.4), which the FP32
path must reproduce within 2 % of the FP64 oracle.  The test shows all three parts of
that statement on one chaotic run: the FP32 state has decorrelated from the oracle's by
the start of the averaging window, its time-averaged flux is within 2 % of the
oracle's, and 2 % lies above the spread of time averages between FP64 trajectories of
the same configuration that differ only by an initial perturbation (the noise floor of
the criterion).  The FP64 GPU path tracks the oracle pointwise over the whole run."""
import numpy as np
import pytest

from parity import log

pytestmark = pytest.mark.gpu

# 256 x 256 pool filled with liquid above a 25-row heater, sites every 32 columns, wall
# superheat 0.15 Tc (Ja = 0.17), g = 3e-5: nucleate boiling with bubbles leaving
# through the outlet.  FP32 and FP64 states are O(0.1) apart from about step 16000.
N0, N1 = 16000, 36000  # averaging window [N0, N1)


def _case(prec, perturb=0.0, seed=0):
    from paper_1812_10375_amd import scenarios as S
    sc = S.pool_boiling(nx=256, ny=256, heater_rows=25, superheat=0.15, g=3e-5, site_spacing=32,
                        liquid_fraction=1.0, seed=0, precision=prec)
    if perturb:
        rng = np.random.default_rng(seed)
        sc["rho0"] = sc["rho0"] * (1.0 + perturb * rng.uniform(-1.0, 1.0, sc["rho0"].shape))
    return sc


def _run_gpu(sc):
    from paper_1812_10375_amd.lbm import Lattice
    lat = Lattice(sc)
    lat.step(N0)
    o0 = lat.observe()
    r0 = lat.read("rho")
    lat.step(N1 - N0)
    o1 = lat.observe()
    r1 = lat.read("rho")
    lat.close()
    return o0, o1, r0, r1


def test_time_averaged_wall_heat_flux_once_boiling_is_chaotic():
    from oracle.lbm import OracleSim
    from paper_1812_10375_amd.surrogate import window_stats
    log("[chaos] oracle: 256 x 256 + 25, %d steps" % N1)
    orc = OracleSim(_case("f64"))
    assert orc.step(N0) == 0
    oo0, ro0 = orc.observe(), orc.field("rho")
    assert orc.step(N1 - N0) == 0
    oo1, ro1 = orc.observe(), orc.field("rho")
    q_orc = window_stats(oo0, oo1)[0]

    def rel(o0, o1):
        return window_stats(o0, o1)[0] / q_orc - 1.0

    # FP32: decorrelated from the oracle at the window start, within 2 % on the average
    g0, g1, r0, r1 = _run_gpu(_case("f32"))
    drift0 = np.abs(r0 - ro0).max() / 6.5
    drift1 = np.abs(r1 - ro1).max() / 6.5
    d32 = rel(g0, g1)
    # FP64 on the GPU: the oracle's trajectory, pointwise
    h0, h1, s0, s1 = _run_gpu(_case("f64"))
    track = max(np.abs(s0 - ro0).max(), np.abs(s1 - ro1).max()) / 6.5
    d64 = rel(h0, h1)
    # the criterion's noise floor: FP64 trajectories of the same configuration whose
    # initial densities differ by 1e-12 stay together (the deterministic floor); with a
    # 1e-3 difference (damped as sound before nucleation, but enough to shift it) they
    # decorrelate as the FP32 run does, and the spread of their time averages is the
    # statistical floor
    p0, p1, _, _ = _run_gpu(_case("f64", 1e-12, seed=1))
    floor_det = abs(rel(p0, p1))
    floor_stat, apart = 0.0, []
    for seed in (1, 2, 3):
        a0, a1, ra, _ = _run_gpu(_case("f64", 1e-3, seed=seed))
        assert a1["status"] == 0 and a1["error_flags"] == 0
        floor_stat = max(floor_stat, abs(rel(a0, a1)))
        apart.append(np.abs(ra - ro0).max() / 6.5)
    log("[chaos] q_bar oracle %.6e; FP32 %+.3e (max|drho|/rho_l %.2f at step %d, %.2f at %d); FP64 GPU %+.1e "
        "(tracks the oracle to %.1e); floor: 1e-12 perturbation %.1e, decorrelated FP64 runs %.3e (apart by %s "
        "at step %d)" % (q_orc, d32, drift0, N0, drift1, N1, d64, track, floor_det, floor_stat,
                         ", ".join("%.2f" % a for a in apart), N0))
    for o in (g1, h1, p1):
        assert o["status"] == 0 and o["error_flags"] == 0
    assert drift0 >= 0.05 and drift1 >= 0.05, "the FP32 run has not decorrelated"
    assert abs(d32) <= 0.02
    assert track <= 1e-8 and abs(d64) <= 1e-8
    assert floor_det <= 1e-8
    assert max(apart) >= 0.01, "no floor run decorrelated"
    assert floor_stat < 0.02  # the 2 % criterion lies above the statistical noise floor


def test_full_length_pool_boiling_run():
    # the 1024 x 1024 + 25 pool-boiling configuration for its full 100k steps, from the
    # paper's all-liquid initial state (Sec. 4.2): bubbles nucleate, rise and leave
    # through the convective outlet without the state going non-finite
    from paper_1812_10375_amd import scenarios as S
    from paper_1812_10375_amd.lbm import Lattice
    sc = S.pool_boiling(nx=1024, ny=1024, liquid_fraction=1.0)
    lat = Lattice(sc)
    m0 = None
    for chunk in range(10):
        lat.step(10000)
        o = lat.observe()
        m0 = o["mass"] if m0 is None else m0
        log("[long] step %d q_bottom_mean %.4e mass %.6e max_speed %.3e" % (
            o["step"], o["q_bottom_mean"], o["mass"], o["max_speed"]))
        assert o["status"] == 0 and o["error_flags"] == 0
        assert o["max_speed"] < 0.3 and o["q_bottom_mean"] > 0
    assert 0.9 * m0 < o["mass"] <= m0
