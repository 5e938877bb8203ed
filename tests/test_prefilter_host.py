"""Host-side selection logic of the pre-filter workflow (no GPU): ranks, recall curves and the
calibration of the docked fraction, the checkpoint directory and the failure hook."""
import os

import numpy as np
import pytest

from paper_2304_09953_amd import prefilter as PF


def test_ranks_break_ties_by_id():
    keys = np.array([3.0, 1.0, 3.0, 1.0, np.inf])
    assert PF.ranks(keys).tolist() == [2, 0, 3, 1, 4]
    assert PF.ranks(keys, np.array([9, 8, 7, 6, 5])).tolist() == [3, 1, 2, 0, 4]


def test_recall_curve_counts_the_kept_share_of_the_true_top():
    rng = np.random.default_rng(0)
    true = rng.normal(size=1000)
    perfect = PF.ranks(true)                      # selection order = true order
    c = PF.recall_curve(perfect, true, [0.005, 0.01, 0.02], 1000)
    assert c == {0.005: 0.5, 0.01: 1.0, 0.02: 1.0}
    worst = PF.ranks(-true)
    assert PF.recall_curve(worst, true, [0.5, 0.99, 1.0], 1000) == {0.5: 0.0, 0.99: 0.0, 1.0: 1.0}
    # a sample of a larger library: ranks are library-wide
    c = PF.recall_curve(np.arange(0, 2000, 2), true, [0.01], 2000)
    top = np.argsort(true, kind="stable")[:10]
    assert c[0.01] == np.mean(2 * top < 20)


def test_calibrate_fraction():
    rng = np.random.default_rng(1)
    true = rng.normal(size=4000)
    assert PF.calibrate_fraction(true, true, 0.95) == 0.01
    noisy = true + rng.normal(scale=0.3, size=4000)
    f = PF.calibrate_fraction(noisy, true, 0.95)
    assert 0.01 < f < 1.0
    r = PF.ranks(noisy)
    assert PF.recall_curve(r, true, [f], 4000)[f] >= 0.95
    assert list(PF.recall_curve(r, true, [f - 0.005], 4000).values())[0] < 0.95
    assert PF.calibrate_fraction(-true, true, 0.95) == 1.0


def test_cascade_recall_and_its_calibration():
    rng = np.random.default_rng(2)
    n = 2000
    true = rng.normal(size=n)
    # a perfect budgeted docking: the pool alone decides, and the final cut keeps all of the top it holds
    pred = true + rng.normal(scale=0.5, size=n)
    in_pool = PF.ranks(pred) < 400
    best = np.argsort(true, kind="stable")[:20]
    assert PF.cascade_recall(pred, true, true, 0.2, 0.03) == np.mean(in_pool[best])
    # a perfect prediction: the budgeted scores alone decide, within the first 3 %
    cheap = true + rng.normal(scale=0.5, size=n)
    assert PF.cascade_recall(true, cheap, true, 1.0, 0.03) == np.mean(PF.ranks(cheap)[best] < 60)
    # a pool smaller than the final cut keeps only the pool
    assert PF.cascade_recall(true, cheap, true, 0.005, 0.03) == 0.5
    # tie order: equal budgeted scores go to the lower index
    flat = np.zeros(n)
    kept = np.sort(np.flatnonzero(in_pool))[:60]
    assert PF.cascade_recall(pred, flat, true, 0.2, 0.03) == np.mean(np.isin(best, kept))
    # calibration: the smallest pool on the grid that reaches the target, 1.0 when none does
    f = PF.calibrate_cascade(pred, cheap, true, 0.03, 0.8)
    assert 0.03 < f < 1.0
    assert PF.cascade_recall(pred, cheap, true, f, 0.03) >= 0.8
    assert PF.cascade_recall(pred, cheap, true, round(f - 0.01, 3), 0.03) < 0.8
    assert PF.calibrate_cascade(-true, -true, true, 0.03, 0.5) == 1.0


def test_linear_baseline_fits_a_linear_target_and_shrinks_with_the_ridge():
    rng = np.random.default_rng(3)
    F = rng.normal(size=(3000, 40)) * rng.uniform(0.1, 5.0, 40) + rng.normal(size=40)
    F[:, 7] = 2.5  # a constant column carries no information and must not break the fit
    w = rng.normal(size=40)
    y = F @ w + 3.0
    X = rng.normal(size=(500, 40)) * 2.0
    X[:, 7] = 2.5
    # an exact linear target is reproduced away from the training points, intercept included
    got = PF.fit_linear(F, y, ridge=1e-9)(X)
    assert np.allclose(got, X @ w + 3.0, rtol=0, atol=1e-6 * np.abs(X @ w + 3.0).max())
    # the ridge shrinks the weights towards the mean label; noise does not move the intercept
    assert np.allclose(PF.fit_linear(F, y, ridge=1e12)(X), y.mean(), atol=1e-3 * np.abs(y).max())
    noisy = y + rng.normal(scale=0.1, size=len(y))
    fit = PF.fit_linear(F, noisy, ridge=1.0)
    assert abs(np.mean(fit(F)) - noisy.mean()) < 1e-9 * np.abs(noisy).max()
    # with no penalty it is the least-squares fit: the residual is orthogonal to every feature
    r = noisy - PF.fit_linear(F, noisy, ridge=1e-9)(F)
    Fc = F - F.mean(0)
    assert np.all(np.abs(Fc.T @ r) <= 1e-8 * np.linalg.norm(Fc, axis=0) * np.linalg.norm(r) + 1e-12)


def test_checkpoint_round_trip_and_manifest(tmp_path):
    d = str(tmp_path / "ck")
    params = {"kind": "screen", "n_lib": 10, "frac": 0.25, "search": {"n_steps": 8, "starts": "ab"}}
    ck = PF.Checkpoint(d, params)
    assert ck.load("predict_0") is None
    a = np.arange(5, dtype=np.float32)
    ck.save("predict_0", preds=a, n_atoms=np.array([3, 4], np.int16))
    got = PF.Checkpoint(d, dict(params)).load("predict_0")  # a rerun with equal parameters sees it
    assert np.array_equal(got["preds"], a) and got["preds"].dtype == np.float32
    assert got["n_atoms"].tolist() == [3, 4]
    assert sorted(os.listdir(d)) == ["manifest.json", "predict_0.npz"]  # no temporary file left behind
    for key, val in (("frac", 0.5), ("search", {"n_steps": 8, "starts": "ac"})):
        with pytest.raises(ValueError, match="another run"):
            PF.Checkpoint(d, {**params, key: val})
    # a file interrupted before its rename is not taken for a finished unit
    with open(os.path.join(d, "predict_1.npz.tmp.npz"), "wb") as f:
        f.write(b"PK\x03")
    assert PF.Checkpoint(d, params).load("predict_1") is None
    # no directory: nothing is written or found
    none = PF.Checkpoint(None, params)
    none.save("x", a=a)
    assert none.load("x") is None


def test_fail_hook_raises_only_for_the_named_unit(monkeypatch):
    monkeypatch.delenv("LIGATE_FAIL_AT", raising=False)
    PF._fail_hook("predict:0")
    monkeypatch.setenv("LIGATE_FAIL_AT", "dock:2")
    PF._fail_hook("dock:1")
    PF._fail_hook("predict:2")
    with pytest.raises(RuntimeError, match="dock:2"):
        PF._fail_hook("dock:2")
