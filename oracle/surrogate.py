"""FP64 oracle of the learned pre-filter (NumPy).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU-baseline leg use
it; the product path never does.  It shares no code with the HIP kernels.

The pre-filter follows the paper's machine-learning engine (§3.5): a cheap model trained on
data the workflow itself generates (§2, the AI engine) predicts each ligand's docking score so
that only the most promising fraction is docked.

* Features (512 per ligand, 16 rows of 32): row t holds the number of type-t atoms, a 30-bin
  histogram of the distances from type-t atoms to every other atom (0.5 A bins on [1.25, 16.25) A,
  values outside folded into the end bins, so the 1.5 A bond length sits mid-bin; ordered pairs,
  i.e. the per-type-pair histograms summed over the partner type) and the rotatable-bond count;
  then log1p.  Distances are Euclidean norms in FP64 of the FP32 input coordinates (widened
  exactly); a distance equal to an inner edge belongs to the bin above it.  A pair lying within
  EDGE_FLAG (1e-5 A) of an inner edge is reported per row by raw_features_flagged: any
  implementation that rounds the distance differently (FP32, or a squared-distance comparison)
  may put such a pair in either neighbouring bin, and it is the only kind of pair that may
  differ.
* Network: y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, 512 -> 1024 -> 1024 -> 1.  Weights are
  BF16 copies (round to nearest even) of FP32 master weights; the input and both hidden layers
  are stored in BF16; sums are exact here (FP64).  Loss: mean squared error.
* Backward: dy = 2 (y - t) / B.  The gradients at the two hidden layers are operands of the
  backward products (they multiply the stored activations to give the weight gradients, and W2
  to give the gradient one layer down), and every operand of a BF16 product is a BF16 value, so
  they are rounded to BF16 like the forward operands.  Weight gradients are FP64 here.  A pin
  compares this gradient with the exact chain rule (grad_exact) of the same network evaluated on
  BF16-rounded weights and inputs: they differ only by these roundings.
* Adam (Kingma and Ba, 2015) with bias correction, no weight decay.
"""
from __future__ import annotations

import numpy as np

N_ROWS, N_SLOTS, N_BINS = 16, 32, 30
BIN_LO, BIN_W = 1.25, 0.5


# ------------------------------------------------------------------------------------------------
# BF16
# ------------------------------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Rounds to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


# ------------------------------------------------------------------------------------------------
# Features
# ------------------------------------------------------------------------------------------------

EDGE_FLAG = 1e-5  # Angstrom


def raw_features_flagged(ligs, status=None):
    """Per-type counts, distance histograms and rotatable count (before log1p), [n_lig, 512], and
    per (ligand, row) the number of pairs within EDGE_FLAG of an inner bin edge, [n_lig, 16].
    Ligands whose status is not OK, or that hold an atom type >= 16, get all-zero rows."""
    out = np.zeros((ligs.n_lig, N_ROWS, N_SLOTS), dtype=np.float64)
    near = np.zeros((ligs.n_lig, N_ROWS), dtype=np.int64)
    inner = BIN_LO + BIN_W * np.arange(1, N_BINS)  # 1.75 .. 15.75 A
    n_rot = ligs.n_rot
    for l in range(ligs.n_lig):
        if status is not None and status[l] != 0:
            continue
        x, t, _, _ = ligs.ligand(l)
        x = x.astype(np.float64)
        t = t.astype(np.int64)
        n = len(t)
        if n == 0 or t.max() >= N_ROWS:
            continue  # a type without a row: the ligand is not representable, zero features
        out[l, :, 0] = np.bincount(t, minlength=N_ROWS)
        if n > 1:
            ii, jj = np.nonzero(~np.eye(n, dtype=bool))  # ordered pairs i != j
            d = np.sqrt(np.sum((x[ii] - x[jj]) ** 2, axis=1))
            b = np.searchsorted(inner, d, side="right")  # 0 below 1.75 A ... 29 from 15.75 A
            np.add.at(out[l], (t[ii], 1 + b), 1.0)
            flag = np.min(np.abs(d[:, None] - inner[None, :]), axis=1) < EDGE_FLAG
            np.add.at(near[l], t[ii], flag.astype(np.int64))
        out[l, :, N_SLOTS - 1] = n_rot[l]
    return out.reshape(ligs.n_lig, N_ROWS * N_SLOTS), near


def raw_features(ligs, status=None) -> np.ndarray:
    return raw_features_flagged(ligs, status)[0]


def features(ligs, status=None) -> np.ndarray:
    return np.log1p(raw_features(ligs, status))


def feature_stats(F: np.ndarray):
    """Training-set mean and 1/std per feature (population std; a feature whose std is below
    1e-6 is constant and is left unscaled: 1/std = 1)."""
    mean = F.mean(0)
    std = F.std(0)
    istd = np.where(std >= 1e-6, 1.0 / np.maximum(std, 1e-6), 1.0)
    return mean, istd


def normalise(F, mean, istd) -> np.ndarray:
    return (F - mean) * istd


# ------------------------------------------------------------------------------------------------
# MLP
# ------------------------------------------------------------------------------------------------

class Params:
    """Flat FP32 master layout: W1 [h1, d], b1 [h1], W2 [h2, h1], b2 [h2], w3 [h2], b3 [1]."""

    def __init__(self, d=512, h1=1024, h2=1024):
        self.d, self.h1, self.h2 = d, h1, h2
        self.shapes = [("W1", (h1, d)), ("b1", (h1,)), ("W2", (h2, h1)), ("b2", (h2,)), ("w3", (h2,)), ("b3", (1,))]
        self.size = sum(int(np.prod(s)) for _, s in self.shapes)

    def split(self, flat):
        out, o = {}, 0
        for name, s in self.shapes:
            k = int(np.prod(s))
            out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(s)
            o += k
        return out

    def join(self, parts) -> np.ndarray:
        return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in self.shapes])


def forward(P: Params, flat, X):
    """Returns y [B] and the cache (BF16-rounded operands) for backward."""
    p = P.split(flat)
    W1, W2, w3 = bf16_round(p["W1"]), bf16_round(p["W2"]), bf16_round(p["w3"])
    x = bf16_round(X)
    h1 = bf16_round(np.maximum(x @ W1.T + p["b1"], 0.0))
    h2 = bf16_round(np.maximum(h1 @ W2.T + p["b2"], 0.0))
    y = h2 @ w3 + p["b3"][0]
    return y, {"x": x, "h1": h1, "h2": h2, "W1": W1, "W2": W2, "w3": w3}


def loss(y, t) -> float:
    return float(np.mean((y - t) ** 2))


def backward(P: Params, flat, X, t):
    """Loss and gradient (flat, same layout as the master weights)."""
    y, c = forward(P, flat, X)
    B = len(t)
    dy = 2.0 * (y - t) / B
    dh2 = bf16_round(dy[:, None] * c["w3"][None, :] * (c["h2"] > 0))
    dh1 = bf16_round((dh2 @ c["W2"]) * (c["h1"] > 0))
    g = {"w3": c["h2"].T @ dy, "b3": np.array([dy.sum()]),
         "W2": dh2.T @ c["h1"], "b2": dh2.sum(0),
         "W1": dh1.T @ c["x"], "b1": dh1.sum(0)}
    return loss(y, t), P.join(g)


def loss_exact(P: Params, flat, X, t) -> float:
    """The same network without any BF16 rounding (for finite-difference checks of backward)."""
    p = P.split(flat)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return loss(y, t)


def grad_exact(P: Params, flat, X, t) -> np.ndarray:
    """Analytic gradient of loss_exact (chain rule written out, no rounding)."""
    p = P.split(flat)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    dy = 2.0 * (y - t) / len(t)
    dh2 = dy[:, None] * p["w3"][None, :] * (a2 > 0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    return P.join({"w3": h2.T @ dy, "b3": np.array([dy.sum()]), "W2": dh2.T @ h1, "b2": dh2.sum(0),
                   "W1": dh1.T @ X, "b1": dh1.sum(0)})


def adam(flat, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------------------------------------
# Metrics
# ------------------------------------------------------------------------------------------------

def r2(y, t) -> float:
    t = np.asarray(t, dtype=np.float64)
    return float(1.0 - np.sum((np.asarray(y) - t) ** 2) / np.sum((t - t.mean()) ** 2))


def spearman(y, t) -> float:
    """Spearman rank correlation with average ranks for ties."""
    def ranks(a):
        a = np.asarray(a, dtype=np.float64)
        order = np.argsort(a, kind="mergesort")
        r = np.empty(len(a))
        r[order] = np.arange(len(a), dtype=np.float64)
        sa = a[order]
        i = 0
        while i < len(a):  # average ranks over runs of equal values
            j = i
            while j + 1 < len(a) and sa[j + 1] == sa[i]:
                j += 1
            if j > i:
                r[order[i:j + 1]] = 0.5 * (i + j)
            i = j + 1
        return r
    ry, rt = ranks(y), ranks(t)
    ry -= ry.mean()
    rt -= rt.mean()
    return float(np.sum(ry * rt) / np.sqrt(np.sum(ry * ry) * np.sum(rt * rt)))


def recall_at(pred_selected_ids, true_scores, true_ids, frac: float) -> float:
    """|true top `frac` of the sample ∩ selected| / |true top `frac`| (lower score = better)."""
    k = max(1, int(round(frac * len(true_scores))))
    top = set(np.asarray(true_ids)[np.lexsort((true_ids, true_scores))[:k]].tolist())
    return len(top & set(np.asarray(pred_selected_ids).tolist())) / k
