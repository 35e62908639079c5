"""The boiling-curve surrogate against the method it replaces: trained on batched runs
of the LB step, it must answer held-out points within 3 % of plain runs on average
(after falling back to plain runs where its members disagree), agree with the plain per-run form on
the training protocol, and produce points at least 20 times faster than one
single-domain run per point."""
import numpy as np
import pytest

from parity import log

pytestmark = pytest.mark.gpu


def test_batched_points_equal_single_runs():
    from paper_1812_10375_amd import surrogate as SG
    proto = SG.Protocol()
    X = SG.sample_inputs(3, seed=42)
    batched, status = SG.run_plain(X, proto)
    assert not status.any()
    for i in range(3):
        one = SG.run_plain_single(X[i], proto)
        assert np.allclose(one, batched[i], rtol=1e-3), (i, one, batched[i])


def test_surrogate_error_and_gain_over_plain_runs():
    from paper_1812_10375_amd import surrogate as SG
    proto = SG.Protocol()
    Xh = SG.sample_inputs(16, seed=99)
    t_single = np.median([SG.timed(SG.run_plain_single, Xh[i], proto)[1] for i in range(3)])
    X = SG.sample_inputs(1024, seed=1)
    (Y, status), t_data = SG.timed(SG.run_plain, X, proto)
    assert not status.any()
    sur = SG.Surrogate(members=4, seed=3)
    loss, t_train = SG.timed(sur.fit, X, Y, 2500)
    Xq = SG.sample_inputs(4096, seed=5)
    (vals, fall), t_query = SG.timed(SG.boiling_curve, sur, Xq, proto, 0.01)
    Yh, _ = SG.run_plain(Xh, proto)
    vh, fh = SG.boiling_curve(sur, Xh, proto, 0.01)
    err = np.abs(vh[:, 0] - Yh[:, 0]) / Yh[:, 0]
    # without the network: the held-out points predicted by the nearest training run
    d = np.linalg.norm(SG.Surrogate.scale(Xh)[:, None] - SG.Surrogate.scale(X)[None], axis=2)
    err_nn = np.abs(Y[d.argmin(1), 0] - Yh[:, 0]) / Yh[:, 0]
    gain = len(Xq) / (t_data + t_train + t_query) * t_single
    log("[surrogate] losses %s held-out err mean %.4f max %.4f (nearest run: %.4f / %.4f), fallback %d/%d, "
        "gain %.1fx (single %.3fs data %.2fs train %.2fs query %.2fs)" % (
            np.round(loss, 4), err.mean(), err.max(), err_nn.mean(), err_nn.max(), len(fall), len(Xq), gain,
            t_single, t_data, t_train, t_query))
    # the mean relative error is the criterion; single points near the boiling crisis,
    # where the curve turns, can be off by more and are reported
    assert err.mean() <= 0.03 and err.max() <= 0.10
    assert err.mean() < err_nn.mean()
    assert gain >= 20
