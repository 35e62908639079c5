"""Host logic of the boiling-curve workflow that needs no GPU: the window statistics
unwound from two running (Welford) records, the input sampling and the protocol."""
import numpy as np
import pytest

from paper_1812_10375_amd import surrogate as SG


def _running(q, n):
    """What an observation after n steps reports: the mean and the population variance
    of the first n per-step fluxes."""
    return {"step": n, "q_bottom_mean": float(np.mean(q[:n])) if n else 0.0,
            "q_bottom_var": float(np.var(q[:n])) if n else 0.0}


@pytest.mark.parametrize("n0,n1", [(0, 500), (200, 500), (499, 500), (1, 2)])
def test_window_stats_equal_the_statistics_of_the_window(n0, n1):
    rng = np.random.default_rng(9)
    q = 1e-3 * (1.0 + 0.3 * rng.standard_normal(500)) + np.linspace(0, 2e-4, 500)
    m, v = SG.window_stats(_running(q, n0), _running(q, n1))
    assert m == pytest.approx(np.mean(q[n0:n1]), rel=1e-12, abs=1e-18)
    assert v == pytest.approx(np.var(q[n0:n1]), rel=1e-8, abs=1e-20)


def test_sampled_inputs_lie_in_the_ranges_with_integer_spacing():
    x = SG.sample_inputs(2000, seed=3)
    assert x.shape == (2000, 4)
    assert np.all(x >= SG.RANGES[:, 0]) and np.all(x <= SG.RANGES[:, 1])
    assert np.array_equal(x[:, 1], np.round(x[:, 1]))
    # the first n points of a larger draw are the draw of n points (training sets grow)
    assert np.array_equal(SG.sample_inputs(512, seed=1), SG.sample_inputs(1024, seed=1)[:512])


def test_protocol_cases_and_window():
    p = SG.Protocol()
    assert (p.nx, p.ny, p.heater_rows, p.steps, p.window) == (256, 256, 25, 50000, 50000)
    sc = p.case(np.array([0.1, 32.0, 0.5, 3e-5]))
    assert sc["nx"] == 256 and sc["ny"] == 256 and sc["heater_rows"] == 25
    assert sc["Gw0"] == 0.5 and sc["g"] == 3e-5
    assert np.all(sc["rho0"] == sc["rho0"].max())  # the pool starts filled with liquid
    with pytest.raises(ValueError):
        SG.Protocol(steps=100, window=200)
