"""Pins of the pre-filter oracle: library routines, closed forms and finite differences."""
import numpy as np
import pytest
import torch
from scipy.spatial.distance import pdist, squareform
from scipy.stats import spearmanr

from oracle import surrogate as S
from paper_2304_09953_amd import inputs as I

RNG = np.random.default_rng(99)


def test_bf16_round_matches_torch():
    x = np.concatenate([RNG.normal(size=5000) * 10 ** RNG.uniform(-6, 6, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(x), ref)
    assert S.bf16_round([1.0 + 2 ** -8])[0] == 1.0  # a tie rounds to even


def test_features_match_numpy_histograms():
    ligs = I.make_ligands(40, I.DIST_HEAVY_TAIL, 16, stream="test")
    F, near = S.raw_features_flagged(ligs)
    F = F.reshape(-1, 16, 32)
    edges = np.r_[-np.inf, 1.25 + 0.5 * np.arange(1, 30), np.inf]
    n_pairs = 0
    for l in range(ligs.n_lig):
        x, t, _, r = ligs.ligand(l)
        n = len(t)
        n_pairs += n * (n - 1)
        D = squareform(pdist(x.astype(np.float64)))
        assert np.array_equal(F[l, :, 0], np.bincount(t, minlength=16))
        assert np.all(F[l, :, 31] == r.sum())
        for ty in range(16):
            rows = np.flatnonzero(t == ty)
            d = np.concatenate([np.delete(D[i], i) for i in rows]) if len(rows) else np.zeros(0)
            h, _ = np.histogram(d, bins=edges)
            # only a pair within 1e-5 A of an edge may fall on the other side (library rounding)
            assert np.abs(F[l, ty, 1:31] - h).sum() <= 2 * near[l, ty]
            assert near[l, ty] == np.sum(np.min(np.abs(d[:, None] - edges[None, 1:-1]), axis=1) < 1e-5)
        assert F[l, :, 1:31].sum() == n * (n - 1)
    # flagged pairs are rare: they cannot hide a wrong binning rule
    assert near.sum() <= 1e-4 * n_pairs


def test_feature_bins_at_and_beside_the_edges():
    """A two-atom ligand at chosen distances: bins of the definition, ends folded in."""
    cases = [(0.9, 0), (1.25, 0), (1.5, 0), (1.7499, 0), (1.75, 1), (2.0, 1), (8.0, 13), (15.7499, 28),
             (15.75, 29), (16.25, 29), (40.0, 29)]
    parts = []
    for d, _ in cases:
        # along x: the coordinates and the distance are exact in FP32 and FP64
        parts.append((np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]], np.float32), np.array([3, 5], np.uint8),
                      np.array([[0, 1]], np.int32), np.array([0], np.uint8)))
    ligs = I.from_parts(parts, 16)
    F, near = S.raw_features_flagged(ligs)
    F = F.reshape(-1, 16, 32)
    for l, (d, b) in enumerate(cases):
        for ty in (3, 5):
            h = np.zeros(30)
            h[b] = 1
            assert np.array_equal(F[l, ty, 1:31], h), (d, ty)
        assert near[l].sum() == (2 if d in (1.75, 15.75) else 0)


def test_unrepresentable_types_give_zero_rows():
    parts = [(np.array([[0, 0, 0], [1.5, 0, 0]], np.float32), np.array([3, 17], np.uint8),
              np.array([[0, 1]], np.int32), np.array([0], np.uint8)),
             (np.array([[0, 0, 0], [1.5, 0, 0]], np.float32), np.array([3, 15], np.uint8),
              np.array([[0, 1]], np.int32), np.array([0], np.uint8))]
    F = S.raw_features(I.from_parts(parts, 32))
    assert np.all(F[0] == 0) and F[1].sum() == 4


def test_features_are_permutation_invariant():
    ligs = I.make_ligands(5, I.DIST_DRUGLIKE, 16, stream="test")
    parts = []
    for l in range(5):
        x, t, b, r = ligs.ligand(l)
        p = RNG.permutation(len(t))
        inv = np.argsort(p)
        parts.append((x[p], t[p], inv[b], r))
    perm = I.from_parts(parts, 16)
    assert np.array_equal(S.raw_features(ligs), S.raw_features(perm))


def test_status_rows_are_zero():
    ligs = I.make_ligands(4, I.DIST_DRUGLIKE, 16, stream="test")
    F = S.features(ligs, status=np.array([0, 3, 0, 1]))
    assert np.all(F[1] == 0) and np.all(F[3] == 0) and F[0].sum() > 0


def test_backward_matches_finite_differences():
    P = S.Params(6, 5, 4)
    flat = RNG.normal(size=P.size) * 0.7
    X = RNG.normal(size=(9, 6))
    t = RNG.normal(size=9)
    g = S.grad_exact(P, flat, X, t)
    h = 1e-6
    fd = np.zeros(P.size)
    for i in range(P.size):
        e = np.zeros(P.size)
        e[i] = h
        fd[i] = (S.loss_exact(P, flat + e, X, t) - S.loss_exact(P, flat - e, X, t)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_bf16_backward_tracks_the_exact_gradient():
    P = S.Params(64, 48, 32)
    flat = RNG.normal(size=P.size) * 0.2
    X = RNG.normal(size=(40, 64))
    t = RNG.normal(size=40)
    _, g = S.backward(P, flat, X, t)
    ge = S.grad_exact(P, flat, X, t)
    # BF16 storage of inputs, activations and their gradients costs a few percent; a wrong term costs O(1)
    assert np.linalg.norm(g - ge) / np.linalg.norm(ge) < 0.1
    # with weights and inputs already on the BF16 grid, the forward pass only rounds activations
    fb = S.bf16_round(flat)
    y, _ = S.forward(P, fb, S.bf16_round(X))
    p = P.split(fb)
    h1 = np.maximum(S.bf16_round(X) @ p["W1"].T + p["b1"], 0)
    assert np.allclose(y, S.bf16_round(np.maximum(S.bf16_round(h1) @ p["W2"].T + p["b2"], 0)) @ p["w3"] + p["b3"][0])


def test_bf16_backward_at_full_width_equals_the_exact_chain_rule_on_bf16_values():
    """512-1024-1024, batch 256: weights, inputs and residuals are small integers (sparse +-1
    weights, integer biases, targets an integer away from the output), so every activation and
    every hidden-layer gradient is a short dyadic number that BF16 holds exactly.  The BF16
    backward must then equal the exact chain rule (pinned by finite differences above) to the
    last bit, with about half of the ReLUs active: any dropped term, wrong sign or transposed
    operand shows."""
    d, h1, h2, B = 512, 1024, 1024, 256
    P = S.Params(d, h1, h2)
    rng = np.random.default_rng(5)

    def sparse(rows, cols, nnz):
        W = np.zeros((rows, cols))
        for r in range(rows):
            W[r, rng.choice(cols, nnz, replace=False)] = rng.choice([-1.0, 1.0], nnz)
        return W

    p = {"W1": sparse(h1, d, 8), "b1": rng.integers(-2, 3, h1).astype(np.float64),
         "W2": sparse(h2, h1, 8), "b2": rng.integers(-2, 3, h2).astype(np.float64),
         "w3": rng.choice([-1.0, 1.0], h2), "b3": np.array([3.0])}
    flat = P.join(p)
    X = rng.integers(-1, 2, (B, d)).astype(np.float64)
    y, c = S.forward(P, flat, X)
    t = y - rng.integers(-3, 4, B)  # residuals -3..3: dy = (y - t) / 128 exactly
    assert np.array_equal(c["h1"], np.maximum(X @ p["W1"].T + p["b1"], 0))  # nothing was rounded
    assert 0.3 < np.mean(c["h1"] > 0) < 0.7 and 0.3 < np.mean(c["h2"] > 0) < 0.7
    _, g = S.backward(P, flat, X, t)
    assert np.array_equal(g, S.grad_exact(P, flat, X, t))


def test_adam_first_step_closed_form():
    g = RNG.normal(size=100)
    w = RNG.normal(size=100)
    w1, m, v = S.adam(w, g, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_metrics():
    t = RNG.normal(size=200)
    assert S.r2(t, t) == 1.0
    assert abs(S.r2(np.full(200, t.mean()), t)) < 1e-12
    y = np.round(t + RNG.normal(size=200) * 0.5, 1)  # with ties
    assert S.spearman(y, t) == pytest.approx(spearmanr(y, t).statistic, abs=1e-12)
    assert S.recall_at([5, 3, 9], np.array([0.1, -2, 3, -1]), np.array([9, 3, 7, 5]), 0.5) == 1.0
    assert S.recall_at([5], np.array([0.1, -2, 3, -1]), np.array([9, 3, 7, 5]), 0.5) == 0.5
