"""Learned pre-filter workflow: label, train, predict, select, dock (the paper's §3.5 engines fed
by data the workflow itself generates, §2).

1. Labels: best docking scores of a training library from the GPU screen.
2. Features -> statistics -> normalised BF16 inputs; an ensemble of networks trained with Adam on
   the matrix cores, each stopped early on a validation split.
3. Held-out R^2 and Spearman correlation; the docked fraction is calibrated on the held-out ligands.
4. Filtered screening of a library streamed in chunks: features and predictions for every ligand,
   global top fraction by prediction, docking of the selected ligands only.
5. Recall of the true top 1 % of a fully docked sample.

Training and the streamed pass can checkpoint to a directory: a manifest of the run's parameters,
then one file per finished unit (a member's epoch: weights, Adam moments and early-stopping state; a
library chunk: predictions, or docking scores).  A rerun with the same directory and parameters
resumes after the last finished unit, and its results equal an uninterrupted run's, since every unit
is a pure function of seeded inputs and the state before it.  LIGATE_FAIL_AT makes a run raise before
a named unit (the test hook of that path).

Every computational step of a network runs in the library's kernels, the members' mean included;
this module orders the calls, moves ligand chunks between host and device, and does the host-side
bookkeeping (validation error, ranks and recall).  The one model fitted on the host is the linear
baseline of the ablation (fit_linear): a comparison for the network, never a selection of the workflow.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import inputs as I
from . import pipeline as P
from . import surrogate as SG


def dock_scores(pocket_dev, search_dev, ligs, chunk: int = 100_000, log=None) -> np.ndarray:
    """Best docking score of every ligand (+inf for invalid ones)."""
    out = np.empty(ligs.n_lig, dtype=np.float32)
    for s in range(0, ligs.n_lig, chunk):
        sub = ligs.subset(np.arange(s, min(s + chunk, ligs.n_lig))) if ligs.n_lig > chunk else ligs
        r = P.screen(pocket_dev, P.DeviceLibrary(sub), search_dev)
        out[s:s + sub.n_lig] = r.best_score.cpu().numpy()
        if log:
            log(f"docked {s + sub.n_lig}/{ligs.n_lig}")
    return out


def library_chunk(dist, n_types, first_id: int, n: int, stream: str = "lib"):
    return I.make_ligands(n, dist, n_types, stream=stream, first_id=first_id)


class Checkpoint:
    """Per-chunk results of a streamed pass in a directory, with a manifest of the run's parameters.

    Opening a directory whose manifest differs from `params` raises: a resumed run must be the same run.
    A chunk's arrays are written to a temporary file and renamed, so a file present is complete."""

    def __init__(self, directory: str | None, params: dict):
        self.dir = directory
        if directory is None:
            return
        os.makedirs(directory, exist_ok=True)
        path = os.path.join(directory, "manifest.json")
        if os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
            if old != params:
                raise ValueError(f"checkpoint directory {directory} holds another run: {old} != {params}")
        else:
            with open(path + ".tmp", "w") as f:
                json.dump(params, f, sort_keys=True)
            os.replace(path + ".tmp", path)

    def _path(self, name: str) -> str:
        return os.path.join(self.dir, name + ".npz")

    def load(self, name: str) -> dict | None:
        if self.dir is None or not os.path.exists(self._path(name)):
            return None
        with np.load(self._path(name)) as z:
            return {k: z[k] for k in z.files}

    def save(self, name: str, **arrays) -> None:
        if self.dir is None:
            return
        tmp = self._path(name) + ".tmp.npz"
        np.savez(tmp, **arrays)
        os.replace(tmp, self._path(name))


def _fail_hook(tag: str) -> None:
    """Raises when LIGATE_FAIL_AT names this unit of work: "predict:<chunk>", "dock:<chunk>" or
    "train:<member>:<epoch>" (chunks counted from 0 in library order)."""
    if os.environ.get("LIGATE_FAIL_AT") == tag:
        raise RuntimeError(f"LIGATE_FAIL_AT: injected failure before {tag}")


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


@dataclass
class Surrogate:
    models: list
    mean: torch.Tensor
    istd: torch.Tensor
    y_mean: float
    y_std: float
    metrics: dict = field(default_factory=dict)
    holdout_pred: np.ndarray | None = None  # predicted and docked best scores of the held-out ligands
    holdout_true: np.ndarray | None = None
    holdout_linear: np.ndarray | None = None  # the linear baseline's predictions of the same ligands

    def predict_z(self, xb: torch.Tensor) -> np.ndarray:
        """Mean of the members' outputs (z-scores of the best docking score) for BF16 features, taken
        on the device (surr_average)."""
        ys = torch.stack([m.predict(xb) for m in self.models])
        return SG.average(ys).cpu().numpy().astype(np.float64)

    def save(self, path: str) -> None:
        """Writes the trained filter to an .npz: each member's FP32 master weights and layer sizes, the
        feature normalisation and the score scale (no optimiser state; Model.state holds that)."""
        m0 = self.models[0]
        arrays = {f"member_{i}": m.master.cpu().numpy() for i, m in enumerate(self.models)}
        np.savez(path, **arrays, dims=np.array([m0.d_in, m0.h1, m0.h2, len(self.models)], np.int64),
                 mean=self.mean.cpu().numpy(), istd=self.istd.cpu().numpy(),
                 y=np.array([self.y_mean, self.y_std], np.float64),
                 metrics=np.array(json.dumps(self.metrics, default=float)))

    @classmethod
    def load(cls, path: str, device="cuda") -> "Surrogate":
        """Reads a filter written by save(); its predictions equal the saved filter's bit for bit."""
        with np.load(path, allow_pickle=False) as z:
            d_in, h1, h2, n = (int(v) for v in z["dims"])
            models = [SG.Model(z[f"member_{i}"], d_in, h1, h2, device=device) for i in range(n)]
            y_mean, y_std = (float(v) for v in z["y"])
            return cls(models, torch.as_tensor(z["mean"]).to(device), torch.as_tensor(z["istd"]).to(device),
                       y_mean, y_std, metrics=json.loads(str(z["metrics"])))

    def fingerprint(self) -> str:
        """Hash of the members' weights and the input normalisation (identifies a trained filter)."""
        h = hashlib.sha256()
        for m in self.models:
            h.update(m.master.cpu().numpy().tobytes())
        h.update(self.mean.cpu().numpy().tobytes())
        h.update(self.istd.cpu().numpy().tobytes())
        h.update(np.array([self.y_mean, self.y_std]).tobytes())
        return h.hexdigest()[:16]

    def predict_library(self, lib_dev) -> np.ndarray:
        """Predicted best score of every ligand of a DeviceLibrary, as the ensemble's z-score (a
        monotone map of the score, so rankings are those of the scores); +inf where the ligand's
        status is not OK."""
        _, xb = SG.features(lib_dev, self.mean, self.istd, f32=False, bf16=True)
        z = self.predict_z(xb).astype(np.float32)
        return np.where(lib_dev.status.cpu().numpy() == 0, z, np.float32(np.inf))


def fit_linear(F: np.ndarray, y: np.ndarray, ridge: float = 1.0):
    """Least squares of y on the features with an intercept, the features standardised on F (columns
    with no spread are left out), a ridge penalty on the weights only: the linear model of the
    pre-filter's ablation, on the same features and training ligands as the network.  Host FP64.
    Returns the predictor X -> y."""
    F = np.asarray(F, np.float64)
    mu, sd = F.mean(axis=0), F.std(axis=0)
    use = sd > 0
    Z = (F[:, use] - mu[use]) / sd[use]
    y = np.asarray(y, np.float64)
    y_mean = float(y.mean())  # the intercept: every column of Z sums to zero
    w = np.linalg.solve(Z.T @ Z + ridge * np.eye(Z.shape[1]), Z.T @ (y - y_mean))

    def predict(X):
        X = np.asarray(X, np.float64)
        return ((X[:, use] - mu[use]) / sd[use]) @ w + y_mean
    return predict


def train_surrogate(pocket_dev, search_dev, train_ligs, labels: np.ndarray | None = None, n_holdout: int = 40_000,
                    n_val: int | None = None, members: int = 4, max_epochs: int = 20, batch: int = 1024,
                    lr: float = 1e-3, seed: int = 0, log=None, checkpoint_dir: str | None = None,
                    linear_baseline: bool = False) -> Surrogate:
    """Labels the training library by docking (unless given) and splits it, in order, into training,
    validation (n_val, default n_holdout / 2) and held-out (n_holdout) ligands.  Feature statistics
    come from the training part.  Each of `members` networks (its own seed for the initial weights
    and the sample order) trains for up to max_epochs and keeps the weights of the epoch with the
    lowest validation error (early stopping); the prediction is the members' mean.  Reports
    held-out R^2 and Spearman.  The generated libraries hold valid ligands only.  With
    checkpoint_dir, every finished epoch is kept there and a rerun resumes after the last one.  With
    linear_baseline, fit_linear on the training part's features predicts the held-out ligands too
    (holdout_linear, and its R^2 and Spearman in the metrics)."""
    n_val = n_holdout // 2 if n_val is None else n_val
    t0 = time.perf_counter()
    if labels is None:
        labels = dock_scores(pocket_dev, search_dev, train_ligs, log=log)
    t_label = time.perf_counter() - t0
    lib = P.DeviceLibrary(train_ligs)
    assert np.all(lib.status.cpu().numpy() == 0) and np.all(np.isfinite(labels))
    n_tr = train_ligs.n_lig - n_holdout - n_val
    assert n_tr > 0
    F, _ = SG.features(lib, bf16=False)
    mean, istd = SG.feature_stats(F[:n_tr])
    _, Xb = SG.features(lib, mean, istd, f32=False, bf16=True)
    F_host = F.cpu().numpy() if linear_baseline and n_holdout else None
    del F
    y = labels.astype(np.float64)
    y_mean, y_std = float(y[:n_tr].mean()), float(y[:n_tr].std())
    z = torch.as_tensor(((y - y_mean) / y_std).astype(np.float32), device=Xb.device)
    Xtr, ztr = Xb[:n_tr], z[:n_tr]
    Xva, zva = Xb[n_tr:n_tr + n_val], (y[n_tr:n_tr + n_val] - y_mean) / y_std
    ck = Checkpoint(checkpoint_dir, {"kind": "train", "n_lig": int(train_ligs.n_lig), "n_holdout": n_holdout,
                                     "n_val": n_val, "members": members, "max_epochs": max_epochs, "batch": batch,
                                     "lr": lr, "seed": seed, "labels": _digest(labels, train_ligs.ids)})
    t1 = time.perf_counter()
    models, best_epochs, hist = [], [], []
    for mbr in range(members):
        model = SG.Model(I.mlp_init(seed=seed + mbr))
        best, best_ep, best_w = np.inf, -1, model.master.clone()
        first = 0
        for ep in range(max_epochs - 1, -1, -1):  # resume after the last finished epoch
            done = ck.load(f"train_{mbr}_{ep}")
            if done is not None:
                model.load_state(done)
                best_w.copy_(torch.as_tensor(done["best_w"]).to(best_w.device))
                best, best_ep, first = float(done["best"]), int(done["best_ep"]), ep + 1
                if mbr == 0:
                    hist = done["hist"].tolist()
                break
        for ep in range(first, max_epochs):
            _fail_hook(f"train:{mbr}:{ep}")
            h = SG.train(model, Xtr, ztr, epochs=1, batch=batch, lr=lr, seed=(seed + mbr) * 100003 + ep)
            if mbr == 0:
                hist += h
            if n_val:
                err = float(np.mean((model.predict(Xva).cpu().numpy().astype(np.float64) - zva) ** 2))
                if err < best:
                    best, best_ep = err, ep
                    best_w.copy_(model.master)
            if ck.dir is not None:
                ck.save(f"train_{mbr}_{ep}", **model.state(), best_w=best_w.cpu().numpy(), best=np.array(best),
                        best_ep=np.array(best_ep), hist=np.array(hist if mbr == 0 else [], np.float64))
            if log:
                log(f"member {mbr}, epoch {ep + 1}/{max_epochs}: train loss {h[0]:.4f}" +
                    (f", validation {err:.4f}" if n_val else ""))
        if n_val:
            model.master.copy_(best_w)
            model.cast()
        models.append(model)
        best_epochs.append(best_ep + 1 if n_val else max_epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    s = Surrogate(models, mean, istd, y_mean, y_std)
    metrics = {"n_train": int(n_tr), "n_validation": int(n_val), "n_holdout": int(n_holdout), "members": members,
               "max_epochs": max_epochs, "best_epochs": best_epochs, "batch": batch, "label_seconds": t_label,
               "train_seconds": t_train, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]}
    if n_holdout:
        from scipy.stats import spearmanr
        pred = s.predict_z(Xb[n_tr + n_val:]) * y_std + y_mean
        yh = y[n_tr + n_val:]
        metrics["holdout_r2"] = float(1 - np.sum((pred - yh) ** 2) / np.sum((yh - yh.mean()) ** 2))
        metrics["holdout_spearman"] = float(spearmanr(pred, yh).statistic)
        s.holdout_pred, s.holdout_true = pred, yh
        if F_host is not None:
            t2 = time.perf_counter()
            lin = fit_linear(F_host[:n_tr], y[:n_tr])(F_host[n_tr + n_val:])
            metrics["linear_fit_seconds"] = time.perf_counter() - t2
            metrics["linear_holdout_r2"] = float(1 - np.sum((lin - yh) ** 2) / np.sum((yh - yh.mean()) ** 2))
            metrics["linear_holdout_spearman"] = float(spearmanr(lin, yh).statistic)
            s.holdout_linear = lin
    s.metrics = metrics
    return s


def filtered_screen(sur: Surrogate, pocket_dev, search_dev, dist, n_types: int, n_lib: int, chunk: int, frac: float,
                    stream: str = "lib", sample_every: int = 0, log=None, checkpoint_dir: str | None = None,
                    extra_fracs=(), cascade_search=None, cascade_pools=(), cascade_final: float = 0.03) -> dict:
    """Predicts every ligand of the streamed library and docks the global top `frac` by
    prediction.  With sample_every > 0 the ligands whose id is a multiple of it are also docked in
    full during the same pass (the recall sample; timed separately).  Each fraction in extra_fracs
    is selected from the same predictions and docked on its own, timed on its own
    (out["extra"][f]).

    Cascade (with cascade_search, a cheaper search budget, and cascade_pools): for each pool
    fraction p, the top p by prediction is docked with cascade_search, and the top cascade_final of
    the library by those scores (taken from the pool) is docked in full (out["cascade"][p]).  The
    recall sample is then also docked with cascade_search (out["sample_cheap_scores"]).

    With checkpoint_dir, finished chunks are kept there and skipped on a rerun of the same run.
    Returns ids, scores, timings (timings cover the chunks computed in this call)."""
    params = {"kind": "screen", "n_lib": n_lib, "chunk": chunk, "frac": frac, "stream": stream,
              "sample_every": sample_every, "n_types": n_types, "dist": repr(dist),
              "filter": sur.fingerprint(), "search": search_dev.desc_fields()}
    if extra_fracs:
        params["extra_fracs"] = [float(f) for f in extra_fracs]
    if cascade_search is not None and cascade_pools:
        params["cascade"] = {"search": cascade_search.desc_fields(), "pools": [float(f) for f in cascade_pools],
                             "final": float(cascade_final)}
    cascade = cascade_search is not None and len(cascade_pools) > 0
    ck = Checkpoint(checkpoint_dir, params)
    preds = np.empty(n_lib, dtype=np.float32)
    n_atoms = np.empty(n_lib, dtype=np.int16)
    t_gen = t_pred = t_sample = t_sample_cheap = 0.0
    s_ids, s_scores, s_cheap = [], [], []
    for ci, s in enumerate(range(0, n_lib, chunk)):
        done = ck.load(f"predict_{ci}")
        if done is not None:
            preds[s:s + len(done["preds"])] = done["preds"]
            n_atoms[s:s + len(done["preds"])] = done["n_atoms"]
            if sample_every:
                s_ids.append(done["sample_ids"])
                s_scores.append(done["sample_scores"])
                if cascade:
                    s_cheap.append(done["sample_cheap"])
            continue
        _fail_hook(f"predict:{ci}")
        g0 = time.perf_counter()
        ligs = library_chunk(dist, n_types, s, min(chunk, n_lib - s), stream)
        t_gen += time.perf_counter() - g0
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        preds[s:s + ligs.n_lig] = sur.predict_library(P.DeviceLibrary(ligs))
        t_pred += time.perf_counter() - p0
        n_atoms[s:s + ligs.n_lig] = ligs.n_atoms
        extra = {}
        if sample_every:
            loc = np.flatnonzero(ligs.ids % sample_every == 0)
            sub = ligs.subset(loc)
            torch.cuda.synchronize()
            d0 = time.perf_counter()
            s_scores.append(P.screen(pocket_dev, P.DeviceLibrary(sub), search_dev).best_score.cpu().numpy())
            t_sample += time.perf_counter() - d0
            s_ids.append(sub.ids)
            extra = {"sample_ids": s_ids[-1], "sample_scores": s_scores[-1]}
            if cascade:
                d0 = time.perf_counter()
                s_cheap.append(P.screen(pocket_dev, P.DeviceLibrary(sub), cascade_search).best_score.cpu().numpy())
                t_sample_cheap += time.perf_counter() - d0
                extra["sample_cheap"] = s_cheap[-1]
        e = s + ligs.n_lig
        ck.save(f"predict_{ci}", preds=preds[s:e], n_atoms=n_atoms[s:e], **extra)
        if log:
            log(f"predicted {s + ligs.n_lig}/{n_lib}" + (f", docked sample {sum(map(len, s_ids))}" if sample_every else ""))
    pred_dev = torch.as_tensor(preds, device="cuda")

    def dock_ids(sel: np.ndarray, search, tag: str, what: str):
        """Docks the ligands `sel` (sorted ids) chunk by chunk with `search`; (scores, dock s, gen s)."""
        scores = np.empty(len(sel), dtype=np.float32)
        t_dock = t_g = 0.0
        for ci, s in enumerate(range(0, n_lib, chunk)):
            part = (sel >= s) & (sel < s + chunk)
            if not part.any():
                continue
            done = ck.load(f"dock{tag}_{ci}")
            if done is not None:
                scores[part] = done["scores"]
                continue
            _fail_hook(f"dock{tag}:{ci}")
            g0 = time.perf_counter()
            ligs = library_chunk(dist, n_types, s, min(chunk, n_lib - s), stream).subset(sel[part] - s)
            t_g += time.perf_counter() - g0
            torch.cuda.synchronize()
            d0 = time.perf_counter()
            scores[part] = P.screen(pocket_dev, P.DeviceLibrary(ligs), search).best_score.cpu().numpy()
            t_dock += time.perf_counter() - d0
            ck.save(f"dock{tag}_{ci}", scores=scores[part])
            if log:
                log(f"docked {what} up to id {s + chunk}")
        return scores, t_dock, t_g

    def top_ids(keys_dev: torch.Tensor, k: int, ids_dev: torch.Tensor | None = None):
        """The k lowest keys (ties to the lower id) on the device; (sorted ids, seconds)."""
        p0 = time.perf_counter()
        _, sel_ids = P.topk(keys_dev, k, ids_dev)
        sel = np.sort(sel_ids.cpu().numpy().astype(np.int64))
        return sel, time.perf_counter() - p0

    def select_and_dock(f: float, tag: str):
        """The global top f by prediction, docked chunk by chunk; (ids, scores, select s, dock s, gen s)."""
        sel, t_sel = top_ids(pred_dev, int(round(f * n_lib)))
        scores, t_dock, t_g = dock_ids(sel, search_dev, tag, f"the top {f:.1%} selection")
        return sel, scores, t_sel, t_dock, t_g

    sel, scores, t_sel, t_dock, t_g = select_and_dock(frac, "")
    t_pred += t_sel
    t_gen += t_g
    out = {"selected_ids": sel, "selected_scores": scores, "predictions": preds, "n_atoms": n_atoms,
           "seconds_predict": t_pred,
           "seconds_dock_selected": t_dock, "seconds_generate_on_host": t_gen, "n_selected": len(sel)}
    out["extra"] = {}
    for i, f in enumerate(extra_fracs):
        e_sel, e_scores, e_tsel, e_tdock, e_tg = select_and_dock(float(f), f"x{i}")
        out["extra"][float(f)] = {"selected_ids": e_sel, "selected_scores": e_scores,
                                  "seconds_predict": t_pred - t_sel + e_tsel, "seconds_dock_selected": e_tdock,
                                  "seconds_generate_on_host": e_tg, "n_selected": len(e_sel)}
    out["cascade"] = {}
    if cascade:
        k_final = int(round(cascade_final * n_lib))
        for i, f in enumerate(cascade_pools):
            pool, t_pool_sel = top_ids(pred_dev, int(round(float(f) * n_lib)))
            cheap, t_pool, t_g1 = dock_ids(pool, cascade_search, f"c{i}", f"the top {float(f):.1%} pool (budget)")
            final, t_fin_sel = top_ids(torch.as_tensor(cheap, device="cuda"), min(k_final, len(pool)),
                                       torch.as_tensor(pool.astype(np.int32), device="cuda"))
            full, t_fin, t_g2 = dock_ids(final, search_dev, f"cf{i}", f"the cascade's top {cascade_final:.1%}")
            out["cascade"][float(f)] = {
                "pool_ids": pool, "pool_cheap_scores": cheap, "selected_ids": final, "selected_scores": full,
                "seconds_predict": t_pred - t_sel + t_pool_sel, "seconds_dock_pool": t_pool,
                "seconds_select_final": t_fin_sel, "seconds_dock_selected": t_fin,
                "seconds_generate_on_host": t_g1 + t_g2, "n_pool": len(pool), "n_selected": len(final)}
    if sample_every:
        out.update(sample_ids=np.concatenate(s_ids), sample_scores=np.concatenate(s_scores),
                   seconds_dock_sample=t_sample)
        if cascade:
            out.update(sample_cheap_scores=np.concatenate(s_cheap), seconds_dock_sample_cheap=t_sample_cheap)
    return out


def ranks(keys: np.ndarray, ids: np.ndarray | None = None) -> np.ndarray:
    """Rank of every entry when sorted by key, ties to the lower id (the selection order of dock_topk)."""
    ids = np.arange(len(keys)) if ids is None else ids
    order = np.lexsort((ids, keys))
    r = np.empty(len(keys), dtype=np.int64)
    r[order] = np.arange(len(keys))
    return r


def recall_curve(key_rank: np.ndarray, true_scores: np.ndarray, fracs, n_total: int, top: float = 0.01) -> dict:
    """For a set of docked ligands with known scores and their rank in the full library's selection
    order: the share of the set's true top `top` that a selection of the first f * n_total ligands
    keeps, for each f."""
    k = max(1, int(round(top * len(true_scores))))
    best = np.lexsort((np.arange(len(true_scores)), true_scores))[:k]
    return {float(f): float(np.mean(key_rank[best] < int(round(f * n_total)))) for f in fracs}


def calibrate_fraction(pred: np.ndarray, true: np.ndarray, target: float, top: float = 0.01,
                       grid=np.round(np.arange(0.005, 1.0001, 0.005), 3)) -> float:
    """Smallest selection fraction whose recall of the true top `top` on a docked held-out set reaches
    `target` (1.0 if none does)."""
    r = ranks(pred)
    curve = recall_curve(r, true, grid, len(pred), top)
    for f in grid:
        if curve[float(f)] >= target:
            return float(f)
    return 1.0


def cascade_recall(pred: np.ndarray, cheap: np.ndarray, true: np.ndarray, pool: float, final: float,
                   top: float = 0.01) -> float:
    """Recall of the true top `top` of a docked set when the top `pool` by prediction is docked with a
    cheaper search and the top `final` of the set by those scores (taken from the pool) is kept.
    Ties go to the lower index, as in dock_topk."""
    n = len(true)
    k = max(1, int(round(top * n)))
    best = set(np.lexsort((np.arange(n), true))[:k].tolist())
    in_pool = np.flatnonzero(ranks(pred) < int(round(pool * n)))
    kept = in_pool[np.lexsort((in_pool, cheap[in_pool]))[:int(round(final * n))]]
    return len(best & set(kept.tolist())) / k


def calibrate_cascade(pred: np.ndarray, cheap: np.ndarray, true: np.ndarray, final: float, target: float,
                      top: float = 0.01, grid=np.round(np.arange(0.01, 1.0001, 0.01), 3)) -> float:
    """Smallest pool fraction whose cascade recall on a docked held-out set reaches `target` (1.0 if
    none does)."""
    for f in grid:
        if f >= final and cascade_recall(pred, cheap, true, float(f), final, top) >= target:
            return float(f)
    return 1.0


def recall_top(sample_ids: np.ndarray, sample_scores: np.ndarray, selected_ids: np.ndarray, frac: float = 0.01):
    k = max(1, int(round(frac * len(sample_ids))))
    order = np.lexsort((sample_ids, sample_scores))[:k]
    top = set(sample_ids[order].tolist())
    return len(top & set(selected_ids.tolist())) / k
