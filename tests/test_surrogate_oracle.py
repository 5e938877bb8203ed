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
    ligs = I.make_ligands(12, I.DIST_DRUGLIKE, 16, stream="test")
    F = S.raw_features(ligs).reshape(-1, 16, 32)
    edges = np.r_[-np.inf, 1.25 + 0.5 * np.arange(1, 30), np.inf]
    for l in range(ligs.n_lig):
        x, t, _, r = ligs.ligand(l)
        n = len(t)
        D = squareform(pdist(x.astype(np.float64)))
        assert np.array_equal(F[l, :, 0], np.bincount(t, minlength=16))
        assert np.all(F[l, :, 31] == r.sum())
        for ty in range(16):
            rows = np.flatnonzero(t == ty)
            d = np.concatenate([np.delete(D[i], i) for i in rows]) if len(rows) else np.zeros(0)
            h, _ = np.histogram(d, bins=edges)
            # FP32 squared distances could put a pair within ~1e-6 A of an edge on the other side
            assert np.abs(F[l, ty, 1:31] - h).sum() <= 2
        assert F[l, :, 1:31].sum() == n * (n - 1)


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
