"""Batched step over independent domains: each domain of a batch must evolve exactly as
it does alone (same tile height), in FP64 and in FP32; batches replay from HIP graphs;
the tile-shape autotuner returns one of its candidates and caches it."""
import numpy as np
import pytest

from paper_1812_10375_amd import scenarios as S
from parity import log

pytestmark = pytest.mark.gpu

HIST = 256


def _mixed(prec, rows=16):
    """Domains of uneven sizes, superheats, sites and boundaries."""
    scs = [
        S.pool_boiling(nx=96, ny=64, heater_rows=5, n_sites=2, min_spacing=16, seed=21, precision=prec,
                       superheat=0.08),
        S.film_evaporation(nx=70, ny=50, film=12, superheat=0.05, seed=22, precision=prec),
        S.pool_boiling(nx=130, ny=40, heater_rows=3, n_sites=1, min_spacing=8, seed=23, precision=prec,
                       superheat=0.15),
        S.interface_conduction(nx=8, ny=96, exact_energy=False, steps=10),
    ]
    scs[3]["precision"] = prec
    for sc in scs:
        sc["tile_rows"] = rows
    return scs


def _fields(read):
    return {k: read(k) for k in ("f", "rho", "ux", "uy", "T")}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_domains_evolve_as_they_do_alone(prec):
    from paper_1812_10375_amd.lbm import BatchLattice, Lattice
    scs = _mixed(prec)
    steps = 300
    log("[batch] %d domains %s %d steps" % (len(scs), prec, steps))
    bat = BatchLattice(scs)
    bat.step(steps)
    bobs = bat.observe()
    for i, sc in enumerate(scs):
        one = Lattice(sc)
        one.step(steps)
        oobs = one.observe()
        a = _fields(lambda k: bat.read(i, k))
        b = _fields(one.read)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, k, np.abs(a[k] - b[k]).max())
        # every observed quantity, the running variance of the bottom flux included
        for k in oobs:
            assert bobs[i][k] == oobs[k], (i, k, bobs[i][k], oobs[k])
        assert bobs[i]["step"] == steps
        one.close()


def test_batch_with_shortened_edge_tile_rows():
    # FP32 domains whose energy grids shorten their first and last tile rows (each its
    # own heights) next to a uniform one, in one batch: each evolves as it does alone
    from paper_1812_10375_amd.lbm import BatchLattice, Lattice
    scs = [S.pool_boiling(nx=128, ny=256, heater_rows=25, n_sites=2, min_spacing=32, seed=5),
           S.pool_boiling(nx=96, ny=300, heater_rows=12, n_sites=2, min_spacing=32, seed=6, superheat=0.2),
           S.film_evaporation(nx=70, ny=50, film=12, superheat=0.05, seed=22, precision="f32")]
    for sc, rows in zip(scs, (44, 40, 16)):
        sc["tile_rows"] = rows
    bat = BatchLattice(scs)
    bat.step(200)
    bobs = bat.observe()
    for i, sc in enumerate(scs):
        one = Lattice(sc)
        one.step(200)
        oobs = one.observe()
        for k in ("rho", "T"):
            assert np.array_equal(bat.read(i, k), one.read(k)), (i, k)
        for k in oobs:
            assert bobs[i][k] == oobs[k], (i, k, bobs[i][k], oobs[k])
        one.close()
    bat.close()


def test_batch_domain_against_the_oracle():
    from oracle.lbm import OracleSim
    from paper_1812_10375_amd.lbm import BatchLattice
    scs = _mixed("f64")
    bat = BatchLattice(scs)
    bat.step(100)
    bat.observe()
    for i in (0, 2):
        orc = OracleSim(scs[i])
        assert orc.step(100) == 0
        for k in ("rho", "T"):
            g, o = bat.read(i, k), orc.field(k)
            assert np.abs(g - o).max() / np.abs(o).max() < 1e-12, (i, k)


def test_batch_graph_replay_matches_eager():
    import torch
    from paper_1812_10375_amd.lbm import BatchLattice
    scs = _mixed("f32")
    eager = BatchLattice(scs)
    want = []
    for _ in range(2):
        eager.step(HIST)
        want.append((eager.observe(), [eager.read(i, "T") for i in range(len(scs))]))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    bat = BatchLattice(scs, stream=s)
    bat.observe()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bat.step(HIST)
    for r in range(2):
        with torch.cuda.stream(s):
            g.replay()
        obs = bat.observe()
        wo, wT = want[r]
        for i in range(len(scs)):
            assert obs[i]["step"] == (r + 1) * HIST
            assert np.array_equal(bat.read(i, "T"), wT[i]), (r, i)
            assert obs[i]["energy"] == wo[i]["energy"]


def test_autotuner_picks_a_candidate_and_caches_it():
    from paper_1812_10375_amd.lbm import autotune_tile_rows
    scs = _mixed("f32", rows=0)
    rows, ms = autotune_tile_rows(scs, steps=5)
    log("[batch] autotune rows=%d ms=%.4f" % (rows, ms))
    assert rows in (8, 12, 16, 20, 24, 32, 40, 48)
    assert ms > 0
    assert autotune_tile_rows(scs, steps=5) == (rows, ms)


def test_shape_autotuner_per_size_class_and_launch_mode():
    # the batch tuner returns a candidate height per domain, one per size class; the
    # one-domain tuner also picks the launch mode; runs with the tuned shapes agree with
    # the default shapes to FP32 rounding (tiles away from the boundaries evaluate the
    # coefficients in their all-fluid form, so the FP32 fields follow the tile shape in
    # their last bits)
    from paper_1812_10375_amd.lbm import BatchLattice, Lattice, autotune
    scs = _mixed("f32", rows=0)
    tuned, ms = autotune(scs, steps=5)
    log("[batch] shape autotune rows=%s ms=%.4f" % ([sc["tile_rows"] for sc in tuned], ms))
    assert ms > 0 and all(sc["tile_rows"] in (8, 12, 16, 20, 24, 32, 40, 48) for sc in tuned)
    cls = {}
    for sc in tuned:
        assert cls.setdefault((sc["nx"], sc["ny"], sc["heater_rows"]), sc["tile_rows"]) == sc["tile_rows"]
    again, ms2 = autotune(scs, steps=5)
    assert ms2 == ms and [sc["tile_rows"] for sc in again] == [sc["tile_rows"] for sc in tuned]
    ref, got = BatchLattice(scs), BatchLattice(tuned)
    ref.step(40)
    got.step(40)
    for i in range(len(scs)):
        for k in ("f", "T"):
            a, b = ref.read(i, k), got.read(i, k)
            assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max(), (i, k)
    ref.close()
    got.close()
    one = S.pool_boiling(nx=256, ny=128, heater_rows=8, n_sites=2, min_spacing=32, seed=5, precision="f32")
    (t1,), ms1 = autotune([one], steps=5)
    log("[batch] one-domain autotune rows=%d flags=%s ms=%.4f" % (t1["tile_rows"], t1["flags"], ms1))
    assert len({"one_launch", "two_launches"} & set(t1["flags"])) == 1
    assert t1["tile_rows"] in (0, 8, 12, 16, 20, 24, 32, 40, 48)
    a, b = Lattice(one), Lattice(t1)
    a.step(40)
    b.step(40)
    for k in ("f", "T"):
        x, y = a.read(k), b.read(k)
        assert np.abs(x - y).max() <= 1e-5 * np.abs(x).max(), k
    a.close()
    b.close()
