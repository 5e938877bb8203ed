"""Bayesian tuning of the search's quality knobs.

The paper tunes the docking engine's quality/performance knobs with a Bayesian optimiser (§3.3,
LiGen autotuning: 11 knobs and more than 6e7 configurations, explored by a method aimed at the
cheapest configuration of a recurring, constrained job).  Here the knobs are the number of
quaternions Q, of translations T and their radius, of torsion steps S, of greedy passes, of swept
starts (sweep_top) and of torsion restarts per rigid start (which the search runs only over every
start, so they exclude sweep_top): about 4.5e4 configurations, too many to screen them all.  The
constraint is the recall of a reference ranking's top fraction on a sample library, the cost the
screen's time per ligand.  The model is a Gaussian process per objective (log time, recall) over
the knobs scaled to [0, 1] (log2 axes for the counts, a linear axis for the radius); the next
configuration maximises expected improvement of the time weighted by the probability that the
recall constraint holds.  Candidates are the discrete grid of knob values; every evaluation is a
real screen (ScreenObjective, or the caller's `evaluate`).  Host-side logic only: it orders screens.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

SPACE = {"n_quat": (16, 24, 32, 48, 64, 96, 128, 192, 256), "n_trans": (4, 8, 12, 16, 24, 32),
         "radius": (2.0, 3.0, 4.0, 5.0), "n_steps": (32, 48, 64, 96, 128, 192, 256), "passes": (1, 2, 3),
         "sweep_top": (0, 16, 32, 64, 128, 256, 512, 1024, 2048), "restarts": (0, 1, 2)}
# the earlier, small space (390 configurations), kept for comparisons where enumeration is affordable
SMALL_SPACE = {"n_quat": (32, 64, 128, 256), "n_trans": (8, 16, 32), "n_steps": (64, 128, 256), "passes": (1, 2),
               "sweep_top": (0, 64, 256, 1024), "restarts": (0, 1, 2)}
LINEAR_KNOBS = ("radius",)


def grid(space: dict = SPACE) -> list[dict]:
    """Every valid combination; a sweep_top reaching Q*T means every start, so it collapses onto 0, and
    restarts go only with every start (sweep_top 0)."""
    out, seen = [], set()
    keys = list(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        c = dict(zip(keys, vals))
        if c.get("sweep_top", 0) >= c["n_quat"] * c["n_trans"]:
            c["sweep_top"] = 0
        if c.get("sweep_top", 0) and c.get("restarts", 0):
            continue
        t = tuple(c[k] for k in keys)
        if t not in seen:
            seen.add(t)
            out.append(c)
    return out


def encode(cfgs: list[dict], space: dict = SPACE) -> np.ndarray:
    """Knob values on a log2 axis scaled to [0, 1] per knob (sweep_top 0, i.e. every start, sits at the
    top of its axis, beyond the largest K; restarts R as 1 + R; the radius on a linear axis)."""
    cols = []
    for k, vals in space.items():
        if k == "sweep_top":
            top = max(vals) * 4
            f = lambda v: math.log2(v if v > 0 else top)  # noqa: E731
            lo, hi = math.log2(min(v for v in vals if v > 0)), math.log2(top)
        elif k == "restarts":  # searched start sets 1 + R on the log2 axis
            f = lambda v: math.log2(1 + v)  # noqa: E731
            lo, hi = math.log2(1 + min(vals)), math.log2(1 + max(vals))
        elif k in LINEAR_KNOBS:
            f, lo, hi = float, float(min(vals)), float(max(vals))
        else:
            f, lo, hi = math.log2, math.log2(min(vals)), math.log2(max(vals))
        cols.append([(f(c[k]) - lo) / (hi - lo) if hi > lo else 0.0 for c in cfgs])
    return np.array(cols, dtype=np.float64).T


class GP:
    """Gaussian process with a squared-exponential kernel, fixed length scale, standardised targets."""

    def __init__(self, length: float = 0.4, noise: float = 1e-4):
        self.length, self.noise = length, noise

    def _k(self, A, B):
        d2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
        return np.exp(-0.5 * d2 / self.length ** 2)

    def fit(self, X: np.ndarray, y: np.ndarray) -> "GP":
        self.X = X
        self.mu, self.sd = float(y.mean()), float(y.std()) or 1.0
        z = (y - self.mu) / self.sd
        K = self._k(X, X) + self.noise * np.eye(len(X))
        self.L = np.linalg.cholesky(K)
        self.alpha = np.linalg.solve(self.L.T, np.linalg.solve(self.L, z))
        return self

    def predict(self, Xs: np.ndarray):
        Ks = self._k(Xs, self.X)
        m = Ks @ self.alpha
        v = np.linalg.solve(self.L, Ks.T)
        var = np.maximum(1.0 - (v * v).sum(0), 1e-12)
        return self.mu + self.sd * m, self.sd * np.sqrt(var)


def _norm_cdf(z):
    from scipy.stats import norm
    return norm.cdf(z)


def _norm_pdf(z):
    from scipy.stats import norm
    return norm.pdf(z)


def constrained_ei(mu_c, sd_c, best_c, mu_r, sd_r, target):
    """Expected improvement of the cost below best_c (+inf: none feasible yet, then the probability of
    feasibility alone) times the probability that the recall reaches target."""
    pf = _norm_cdf((mu_r - target) / sd_r)
    if not np.isfinite(best_c):
        return pf
    z = (best_c - mu_c) / sd_c
    return ((best_c - mu_c) * _norm_cdf(z) + sd_c * _norm_pdf(z)) * pf


def optimize(evaluate, target: float, space: dict = SPACE, n_init: int = 6, n_iter: int = 20, seed: int = 0,
             log=None) -> dict:
    """Minimises cost subject to recall >= target.  evaluate(cfg) -> (cost, recall); cost > 0.
    Returns the history and the best feasible configuration found."""
    cands = grid(space)
    X = encode(cands, space)
    rng = np.random.default_rng(seed)
    done, hist = [], []

    def run(i):
        cost, rec = evaluate(cands[i])
        done.append(i)
        hist.append({"cfg": cands[i], "cost": float(cost), "recall": float(rec)})
        if log:
            log(f"knobs {cands[i]}: cost {cost:.4g}, recall {rec:.3f}")

    for i in rng.choice(len(cands), size=min(n_init, len(cands)), replace=False):
        run(int(i))
    for _ in range(n_iter):
        if len(done) == len(cands):
            break
        Xd = X[done]
        c = np.log(np.array([h["cost"] for h in hist]))
        r = np.array([h["recall"] for h in hist])
        feas = r >= target
        best_c = c[feas].min() if feas.any() else np.inf
        gp_c, gp_r = GP().fit(Xd, c), GP().fit(Xd, r)
        rest = np.setdiff1d(np.arange(len(cands)), done)
        mc, sc = gp_c.predict(X[rest])
        mr, sr = gp_r.predict(X[rest])
        acq = constrained_ei(mc, sc, best_c, mr, sr, target)
        run(int(rest[int(np.argmax(acq))]))
    return {"history": hist, "best": best_feasible(hist, target)}


def random_search(evaluate, target: float, n: int, space: dict = SPACE, seed: int = 0) -> dict:
    cands = grid(space)
    rng = np.random.default_rng(seed)
    hist = []
    for i in rng.choice(len(cands), size=min(n, len(cands)), replace=False):
        cost, rec = evaluate(cands[int(i)])
        hist.append({"cfg": cands[int(i)], "cost": float(cost), "recall": float(rec)})
    return {"history": hist, "best": best_feasible(hist, target)}


def best_feasible(hist: list[dict], target: float):
    ok = [h for h in hist if h["recall"] >= target]
    return min(ok, key=lambda h: h["cost"]) if ok else None


class ScreenObjective:
    """(cost, recall) of a knob configuration by real screens: cost = seconds per 1M ligands of the
    screen (HIP events around a second run of the same screen), recall = the share of the reference
    search's top fraction of the library (ties to the lower ligand) that the configuration's own top
    fraction keeps.  Configurations are cached."""

    def __init__(self, pocket_dev, lib_dev, reference, top_frac: float = 0.01, radius: float = 4.0):
        self.dp, self.lib, self.frac, self.radius = pocket_dev, lib_dev, top_frac, radius
        self.cache = {}
        self.ref_seconds, ref = self.screen(reference)
        self.ok = np.isfinite(ref)
        self.ids = np.flatnonzero(self.ok)
        self.k = max(1, int(round(top_frac * self.ok.sum())))
        self.top_ref = set(self._top(ref).tolist())

    def _top(self, best):
        return self.ids[np.lexsort((self.ids, best[self.ok]))[:self.k]]

    def screen(self, srch):
        """Seconds of one screen and the per-ligand best scores."""
        import torch

        from . import pipeline as P
        scr = P.Screener(self.dp, self.lib, P.DeviceSearch(srch))
        scr.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        scr.run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3, scr.best_score.cpu().numpy().astype(np.float64)

    def search_of(self, cfg):
        import dataclasses

        from . import inputs as I
        R = int(cfg.get("restarts", 0))
        base = I.make_search(cfg["n_quat"], cfg["n_trans"], cfg["n_steps"], float(cfg.get("radius", self.radius)),
                             self.dp.pocket.center)
        return dataclasses.replace(base, sweep_top=int(cfg.get("sweep_top", 0)), passes=int(cfg.get("passes", 1)),
                                   restarts=R, init_steps=I.restart_steps(R, cfg["n_steps"]) if R else None)

    def recall_of(self, best) -> float:
        return len(set(self._top(best).tolist()) & self.top_ref) / self.k

    def __call__(self, cfg):
        key = tuple(sorted(cfg.items()))
        if key not in self.cache:
            t, best = self.screen(self.search_of(cfg))
            self.cache[key] = (t / self.lib.n_lig * 1e6, self.recall_of(best))
        return self.cache[key]
