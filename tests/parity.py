"""Shared helpers of the GPU parity tests: run a scenario on the GPU library and on the
oracle from the same seeded inputs and measure their differences."""
import sys

import numpy as np

from paper_1812_10375_amd import scenarios as S


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pair(sc, steps, fields=("rho", "ux", "uy", "T")):
    from oracle.lbm import OracleSim
    from paper_1812_10375_amd.lbm import Lattice
    log("[parity] %s nx=%d ny=%d nh=%d prec=%s steps=%d" % (
        sc.get("name", "?"), sc["nx"], sc["ny"], sc["heater_rows"], sc["precision"], steps))
    gpu = Lattice(sc)
    gpu.step(steps)
    og = gpu.observe()
    orc = OracleSim(sc)
    rc = orc.step(steps)
    assert rc == 0, "oracle flagged an error"
    oo = orc.observe()
    out = {"gpu_obs": og, "orc_obs": oo}
    for f in fields:
        a, b = gpu.read(f), orc.field(f)
        out[f] = (a, b)
    return out, gpu, orc


def errors(res):
    ra, rb = res["rho"]
    Ta, Tb = res["T"]
    ua, ub = res["ux"]
    va, vb = res["uy"]
    umax = max(np.abs(ub).max(), np.abs(vb).max(), 1e-300)
    return {
        "rho": np.abs(ra - rb).max() / S.RHO_L,
        "T": np.abs(Ta - Tb).max() / S.TC,
        "u": max(np.abs(ua - ub).max(), np.abs(va - vb).max()) / umax,
        "umax": umax,
    }
