"""Boiling-curve surrogate built on the LB method.

One boiling-curve point is the time-averaged heat flux through the bottom of the
heater, and its variance over time, for a pool-boiling configuration (Sec. 4.2-4.4).
A point has four inputs: wall superheat, nucleation-site spacing, wall strength G_w0
of Eq. 10 (the contact-angle parameter) and gravity g of Eq. 9.  The plain form runs
the LB method for every point.  This module adds two faster forms:

* batched runs: many points advance together in one batched step;
* a surrogate: an ensemble of small MLPs trained on batched runs of the method, with
  BF16 matrix-core kernels.  A query falls back to batched plain runs where the
  members disagree by more than a threshold, or where the training runs nearest to it
  were predicted worse than that when left out of a member's resample.

Every step of the method runs in the library's kernels.  This module only builds
scenarios, reads observations and moves arrays.
"""
import time

import numpy as np

from . import scenarios as S

# input ranges (superheat in units of T_c, site spacing in lattice units)
RANGES = np.array([[0.02, 0.30], [16.0, 64.0], [0.3, 0.7], [1e-5, 5e-5]])
INPUTS = ("superheat", "site_spacing", "Gw0", "g")


class Protocol:
    """Run protocol of one point: a pool of nx x ny filled with liquid above a heater of
    `heater_rows` rows, `steps` LB steps, statistics over the last `window` steps.

    The default is the smallest domain of the batched pool-boiling workload (256 x 256
    above 25 heater rows) run for that workload's 50k steps, averaged over the whole run:
    the heat a run draws through the heater's bottom per step, and its variance over the
    steps.  At this size the later part of a run is still a transient (the pool keeps
    warming: averages over steps 25k-50k and 25k-150k differ by 32% at the median), so a
    late window is no steadier a boiling-curve value, while the whole-run average is
    deterministic (runs from initial densities perturbed by 1e-3 agree to 0.1% at the
    median) and varies smoothly enough with the inputs to be learnt."""

    def __init__(self, nx=256, ny=256, heater_rows=25, steps=50000, window=50000):
        if not 0 < window <= steps:
            raise ValueError("the window must lie within the run")
        self.nx, self.ny, self.heater_rows = nx, ny, heater_rows
        self.steps, self.window = steps, window

    def describe(self):
        return "%dx%d+%d pool, all liquid, %d steps, statistics over the last %d" % (
            self.nx, self.ny, self.heater_rows, self.steps, self.window)

    def case(self, p, precision="f32"):
        sc = S.pool_boiling(nx=self.nx, ny=self.ny, heater_rows=self.heater_rows, superheat=float(p[0]),
                            g=float(p[3]), site_spacing=int(round(p[1])), Gw0=float(p[2]),
                            liquid_fraction=1.0, seed=0, precision=precision)
        sc["name"] = "point_%.4f_%d_%.3f_%.2e" % (p[0], int(round(p[1])), p[2], p[3])
        return sc


def sample_inputs(n, seed):
    """n points drawn uniformly from RANGES (spacing rounded to an integer)."""
    rng = np.random.default_rng(seed)
    x = RANGES[:, 0] + (RANGES[:, 1] - RANGES[:, 0]) * rng.uniform(size=(n, 4))
    x[:, 1] = np.round(x[:, 1])
    return x


def window_stats(o0, o1):
    """Mean and variance of the bottom heat flux over the steps between two
    observations, from the running (Welford) statistics each one reports."""
    n0, n1 = float(o0["step"]), float(o1["step"])
    nw = n1 - n0
    m0, m1 = o0["q_bottom_mean"], o1["q_bottom_mean"]
    mw = (n1 * m1 - n0 * m0) / nw
    m2 = o1["q_bottom_var"] * n1 - o0["q_bottom_var"] * n0 - (mw - m0) ** 2 * n0 * nw / n1
    return mw, max(m2, 0.0) / nw


def run_plain(points, proto, chunk=512, progress=None):
    """Boiling-curve points by batched runs of the method: returns [n][2] (mean, var)
    and the status of each run.  progress(done, total) is called after every batch."""
    from .lbm import BatchLattice
    points = np.asarray(points, dtype=np.float64).reshape(-1, 4)
    out = np.zeros((len(points), 2))
    status = np.zeros(len(points), dtype=int)
    for a in range(0, len(points), chunk):
        part = points[a:a + chunk]
        bat = BatchLattice([proto.case(p) for p in part])
        bat.step(proto.steps - proto.window)
        o0 = bat.observe(check=False)
        if any(o["status"] for o in o0):
            bat.close()
            raise RuntimeError("a plain run became non-finite before its window")
        bat.step(proto.window)
        o1 = bat.observe(check=False)
        for i, (u, v) in enumerate(zip(o0, o1)):
            out[a + i] = window_stats(u, v)
            status[a + i] = v["error_flags"]
        bat.close()
        if progress:
            progress(a + len(part), len(points))
    return out, status


def run_plain_single(point, proto, tile_rows=0):
    """One boiling-curve point by a single-domain run (the plain per-run form); tile_rows
    as in the library's configuration (0: the automatic tiles of one domain)."""
    from .lbm import Lattice
    sc = proto.case(point)
    sc["tile_rows"] = tile_rows
    lat = Lattice(sc)
    lat.step(proto.steps - proto.window)
    o0 = lat.observe()
    lat.step(proto.window)
    o1 = lat.observe()
    lat.close()
    return np.array(window_stats(o0, o1))


class Surrogate:
    """Ensemble of MLPs on the GPU mapping scaled inputs to the standardised logarithms
    of the heat-flux mean and variance (so that errors are relative).  Each member is
    trained on its own bootstrap resample of the points.  Two estimates of the relative
    error of a prediction come with it:

    * the members' spread of log q (the model's uncertainty);
    * the out-of-bag error of the nearest training runs: each training run is predicted
      by the members whose resample left it out, and a query takes the mean of that
      error over its `k_local` nearest runs in the scaled input space.  This catches
      regions where the members agree but the flux varies faster than the runs resolve
      (near the boiling crisis), which the spread alone misses."""

    def __init__(self, members=4, seed=1, k_local=8):
        self.members, self.seed, self.k_local = members, seed, k_local
        self.net = None

    @staticmethod
    def scale(points):
        p = np.asarray(points, dtype=np.float64).reshape(-1, 4)
        return 2.0 * (p - RANGES[:, 0]) / (RANGES[:, 1] - RANGES[:, 0]) - 1.0

    def fit(self, points, values, steps=4000, lr=2e-3, lr_end=5e-5):
        """Train every member on a bootstrap resample of the points (full batch, Adam,
        cosine-decayed rate), then record every run's out-of-bag error; returns the final
        losses."""
        import torch
        from .mlp import MLPEnsemble
        X = self.scale(points)
        L = np.log(np.maximum(np.asarray(values, dtype=np.float64), 1e-300))
        self.mu, self.sd = L.mean(axis=0), L.std(axis=0)
        self.sd[self.sd == 0] = 1.0
        T = (L - self.mu) / self.sd
        rng = np.random.default_rng(self.seed)
        idx = rng.integers(0, len(X), size=(self.members, len(X)))
        Xd = torch.as_tensor(X[idx], dtype=torch.float32, device="cuda")
        Td = torch.as_tensor(T[idx], dtype=torch.float32, device="cuda")
        self.net = MLPEnsemble(self.members, max(len(X), 16384), params=S.mlp_init_params(self.seed, self.members))
        for it in range(steps):
            r = lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * it / steps))
            self.net.train_step(Xd, Td, r)
        losses = self.net.backward(Xd, Td).cpu().numpy()
        # out-of-bag error of every training run (NaN where every member drew it)
        oob = np.ones((self.members, len(X)), dtype=bool)
        for m in range(self.members):
            oob[m, idx[m]] = False
        Lm = self._members(X)[:, :, 0]
        n_oob = oob.sum(axis=0)
        lo = np.where(oob, Lm, 0.0).sum(axis=0) / np.maximum(n_oob, 1)
        err = np.abs(np.exp(lo - L[:, 0]) - 1.0)
        self.X_train, self.oob_err = X, np.where(n_oob > 0, err, np.nan)
        return losses

    def _members(self, Xs):
        """Every member's logarithms of (q mean, q variance) at scaled inputs: [members][n][2]."""
        outs = []
        for a in range(0, len(Xs), self.net.max_batch):
            outs.append(self.net.forward(Xs[a:a + self.net.max_batch]).cpu().numpy().astype(np.float64))
        return np.concatenate(outs, axis=1) * self.sd + self.mu

    def predict(self, points):
        """Ensemble estimate of (q mean, q variance), the members' spread of log q, and
        the mean out-of-bag error of the nearest training runs."""
        Xq = self.scale(points)
        Y = self._members(Xq)
        vals = np.exp(Y.mean(axis=0))
        local = np.empty(len(Xq))
        for a in range(0, len(Xq), 2048):
            d = np.linalg.norm(Xq[a:a + 2048, None, :] - self.X_train[None], axis=2)
            near = np.argpartition(d, self.k_local - 1, axis=1)[:, :self.k_local]
            local[a:a + 2048] = np.nanmean(self.oob_err[near], axis=1)
        return vals, Y[:, :, 0].std(axis=0), local


def boiling_curve(surrogate, points, proto, threshold=0.05, progress=None):
    """Boiling-curve values for `points`: the surrogate's prediction where both error
    estimates (the members' spread of log q, the out-of-bag error of the nearest runs)
    are within `threshold`, batched plain runs of the method elsewhere."""
    vals, spread, local = surrogate.predict(points)
    fall = np.nonzero((spread > threshold) | (local > threshold))[0]
    if len(fall):
        vals[fall], _ = run_plain(np.asarray(points)[fall], proto, progress=progress)
    return vals, fall


def timed(fn, *a, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn(*a, **kw)
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0
