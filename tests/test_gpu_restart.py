"""Checkpoint and restart: a run interrupted after some steps, saved (populations,
temperature and the run state record) and continued in a fresh context must match the
uninterrupted run bitwise, fields and every observed quantity, in FP64, in FP32 with two
launches per step and in FP32 with the fused launch; across a change of step parity; and
a state record of another configuration is refused."""
import numpy as np
import pytest

from paper_1812_10375_amd import scenarios as S
from parity import log

pytestmark = pytest.mark.gpu


def _scenario(prec, mode):
    sc = S.pool_boiling(nx=96, ny=70, heater_rows=5, n_sites=2, min_spacing=16, seed=11, superheat=0.2,
                        liquid_fraction=0.6, precision=prec)
    if mode:
        sc["flags"] = tuple(sc["flags"]) + (mode,)
    return sc


@pytest.mark.parametrize("prec,mode,cut", [("f64", None, 171), ("f32", "two_launches", 170),
                                           ("f32", "one_launch", 171), ("f32", "one_launch", 300)])
def test_interrupted_run_continues_bitwise(prec, mode, cut):
    from paper_1812_10375_amd.lbm import Lattice
    total = 400
    sc = _scenario(prec, mode)
    log("[restart] %s %s cut at %d of %d" % (prec, mode, cut, total))
    ref = Lattice(sc)
    ref.step(total)
    want = ref.observe()
    want_f = {k: ref.read(k) for k in ("f", "rho", "ux", "uy", "T")}
    ref.close()
    first = Lattice(sc)
    first.step(cut)
    first.observe()
    ck = first.checkpoint()
    first.close()
    # a fresh context of the same configuration, started from another state
    again = Lattice(sc)
    again.step(7)
    again.restore(ck)
    mid = again.observe()
    assert mid["step"] == cut
    again.step(total - cut)
    got = again.observe()
    for k in want_f:
        a = again.read(k)
        assert np.array_equal(a, want_f[k]), (k, np.abs(a - want_f[k]).max())
    for k in want:
        assert got[k] == want[k], (k, got[k], want[k])
    again.close()


def test_state_of_another_configuration_is_refused():
    from paper_1812_10375_amd.lbm import LbmError, Lattice
    a = Lattice(_scenario("f32", None))
    b = Lattice(S.film_evaporation(nx=64, ny=40, film=10, precision="f32"))
    a.step(3)
    rec = a.read_state()
    with pytest.raises(LbmError):
        b.write_state(rec)
    bad = rec.copy()
    bad[:8] = 0  # not a state record
    with pytest.raises(LbmError):
        a.write_state(bad)
    a.close()
    b.close()


@pytest.mark.parametrize("mode", ["one_launch", "two_launches"])
def test_rewind_in_the_same_context(mode):
    # restoring an earlier state into the context that ran past it, then running on,
    # repeats the run bitwise (the fused step's per-tile completion marks count steps
    # and must restart with the restored step)
    from paper_1812_10375_amd.lbm import Lattice
    lat = Lattice(_scenario("f32", mode))
    lat.step(120)
    ck = lat.checkpoint()
    lat.step(200)
    want = lat.observe()
    want_f = {k: lat.read(k) for k in ("f", "T")}
    lat.restore(ck)
    lat.step(200)
    got = lat.observe()
    for k in want_f:
        assert np.array_equal(lat.read(k), want_f[k]), k
    for k in want:
        assert got[k] == want[k], (k, got[k], want[k])
    lat.close()
