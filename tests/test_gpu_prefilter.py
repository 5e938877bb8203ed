"""The learned pre-filter end to end on the GPU: what the trained network gains over selecting
without it, the filtered workflow's selection and docking against plain docking, and runs that fail
at a named unit of work and resume from their checkpoint directory."""
import numpy as np
import pytest
import torch

from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    from paper_2304_09953_amd import prefilter as PF
    W = I.workload("pocket96-lib100k")
    dp, ds = P.DevicePocket(W.pockets[0]), P.DeviceSearch(W.search)
    ligs = I.make_ligands(6000, W.dist, W.n_types, stream="test")
    say("dock 6000 training ligands (full search), train a 2-member ensemble")
    sur = PF.train_surrogate(dp, ds, ligs, n_holdout=1500, n_val=500, members=2, max_epochs=10, batch=256,
                             linear_baseline=True)
    say(f"surrogate metrics {sur.metrics}")
    return P, PF, W, dp, ds, ligs, sur


def test_network_beats_selection_without_it(trained):
    P, PF, W, dp, ds, ligs, sur = trained
    pred, true = sur.holdout_pred, sur.holdout_true
    ho = np.arange(ligs.n_lig - 1500, ligs.n_lig)
    fr = [0.1, 0.25]
    net = PF.recall_curve(PF.ranks(pred), true, fr, len(true), top=0.05)
    big = PF.recall_curve(PF.ranks(-ligs.n_atoms[ho].astype(np.float64)), true, fr, len(true), top=0.05)
    small = PF.recall_curve(PF.ranks(ligs.n_atoms[ho].astype(np.float64)), true, fr, len(true), top=0.05)
    lin = PF.recall_curve(PF.ranks(sur.holdout_linear), true, fr, len(true), top=0.05)
    say(f"recall of the true top 5 %: network {net}, linear model of the same features {lin} (held-out R^2 "
        f"{sur.metrics['linear_holdout_r2']:.3f}), largest first {big}, smallest first {small}, random = f")
    assert sur.holdout_linear.shape == true.shape and np.isfinite(sur.metrics["linear_holdout_r2"])
    assert sur.metrics["holdout_spearman"] > 0.8
    for f in fr:
        assert net[f] >= f + 0.4                       # random selection keeps a share f
        assert net[f] > max(big[f], small[f]) + 0.1    # and the size heuristics less than the network


def test_filtered_screen_selects_by_prediction_and_docks_like_plain(trained):
    P, PF, W, dp, ds, ligs, sur = trained
    say("filtered screen of a 3000-ligand library, top 20 %, every 3rd ligand also docked in full")
    res = PF.filtered_screen(sur, dp, ds, W.dist, W.n_types, 3000, 1000, 0.2, stream="sample", sample_every=3)
    preds = res["predictions"]
    order = np.lexsort((np.arange(3000), preds))
    assert np.array_equal(np.sort(order[:600]), res["selected_ids"])
    lib = I.make_ligands(3000, W.dist, W.n_types, stream="sample")
    plain = P.screen(dp, P.DeviceLibrary(lib), ds).best_score.cpu().numpy()
    assert np.array_equal(res["selected_scores"], plain[res["selected_ids"]])
    assert np.array_equal(res["sample_ids"], np.arange(0, 3000, 3))
    assert np.array_equal(res["sample_scores"], plain[::3])
    # recall from the selection equals the curve read from the prediction ranks
    r = PF.recall_top(res["sample_ids"], res["sample_scores"], res["selected_ids"], 0.05)
    c = PF.recall_curve(PF.ranks(preds)[res["sample_ids"]], res["sample_scores"].astype(np.float64), [0.2], 3000,
                        top=0.05)
    assert r == c[0.2]


def test_cascade_selects_by_budget_scores_and_docks_like_plain(trained):
    import dataclasses
    P, PF, W, dp, ds, ligs, sur = trained
    cs = P.DeviceSearch(dataclasses.replace(W.search, sweep_top=256))
    say("cascade on a 3000-ligand library: top 20 % by prediction docked with the best 256 rigid starts swept, "
        "then the top 3 % by those scores docked in full")
    res = PF.filtered_screen(sur, dp, ds, W.dist, W.n_types, 3000, 1000, 0.1, stream="sample", sample_every=3,
                             cascade_search=cs, cascade_pools=(0.2,), cascade_final=0.03)
    c = res["cascade"][0.2]
    ids = np.arange(3000)
    pool = np.sort(np.lexsort((ids, res["predictions"]))[:600])
    assert np.array_equal(c["pool_ids"], pool)
    lib = I.make_ligands(3000, W.dist, W.n_types, stream="sample")
    cheap = P.screen(dp, P.DeviceLibrary(lib), cs).best_score.cpu().numpy()
    assert np.array_equal(c["pool_cheap_scores"], cheap[pool])
    final = np.sort(pool[np.lexsort((pool, cheap[pool]))[:90]])
    assert np.array_equal(c["selected_ids"], final)
    plain = P.screen(dp, P.DeviceLibrary(lib), ds).best_score.cpu().numpy()
    assert np.array_equal(c["selected_scores"], plain[final])
    assert np.array_equal(res["sample_cheap_scores"], cheap[::3])
    # the held-out form of the same cascade, on all 3000 ligands, reproduces the recall of the selection
    sel = set(final.tolist())
    full_casc = PF.cascade_recall(res["predictions"].astype(np.float64), cheap.astype(np.float64),
                                  plain.astype(np.float64), 0.2, 0.03, top=0.01)
    assert full_casc == np.mean([i in sel for i in np.lexsort((ids, plain))[:30]])


def test_filtered_screen_resumes_after_a_failure(trained, tmp_path, monkeypatch):
    P, PF, W, dp, ds, ligs, sur = trained
    args = (sur, dp, ds, W.dist, W.n_types, 2500, 1000, 0.2)
    kw = dict(stream="tiny", sample_every=4)
    say("filtered screen of 2500 ligands, uninterrupted, then failing before prediction chunk 1 and dock chunk 2")
    ref = PF.filtered_screen(*args, **kw)
    d = str(tmp_path / "screen")
    for tag in ("predict:1", "dock:2"):
        monkeypatch.setenv("LIGATE_FAIL_AT", tag)
        with pytest.raises(RuntimeError, match=tag):
            PF.filtered_screen(*args, **kw, checkpoint_dir=d)
    monkeypatch.delenv("LIGATE_FAIL_AT")
    res = PF.filtered_screen(*args, **kw, checkpoint_dir=d)
    for key in ("selected_ids", "selected_scores", "predictions", "n_atoms", "sample_ids", "sample_scores"):
        assert np.array_equal(res[key], ref[key]), key
    with pytest.raises(ValueError, match="another run"):
        PF.filtered_screen(sur, dp, ds, W.dist, W.n_types, 2500, 1000, 0.3, **kw, checkpoint_dir=d)


def test_training_resumes_after_a_failure(trained, tmp_path, monkeypatch):
    P, PF, W, dp, ds, ligs, sur = trained
    sub = I.make_ligands(3000, W.dist, W.n_types, stream="train")
    labels = PF.dock_scores(dp, ds, sub)
    kw = dict(labels=labels, n_holdout=500, n_val=300, members=2, max_epochs=3, batch=256)
    say("train a 2-member ensemble for 3 epochs, uninterrupted, then failing before member 1's epoch 1")
    ref = PF.train_surrogate(dp, ds, sub, **kw)
    d = str(tmp_path / "train")
    monkeypatch.setenv("LIGATE_FAIL_AT", "train:1:1")
    with pytest.raises(RuntimeError, match="train:1:1"):
        PF.train_surrogate(dp, ds, sub, **kw, checkpoint_dir=d)
    monkeypatch.delenv("LIGATE_FAIL_AT")
    res = PF.train_surrogate(dp, ds, sub, **kw, checkpoint_dir=d)
    for a, b in zip(ref.models, res.models):
        assert torch.equal(a.master, b.master) and torch.equal(a.bf16, b.bf16)
    assert res.metrics["best_epochs"] == ref.metrics["best_epochs"]
    assert res.metrics["loss_first_epoch"] == ref.metrics["loss_first_epoch"]
    assert res.metrics["loss_last_epoch"] == ref.metrics["loss_last_epoch"]
    assert np.array_equal(res.holdout_pred, ref.holdout_pred)


def test_saved_filter_predicts_like_the_trained_one(trained, tmp_path):
    P, PF, W, dp, ds, ligs, sur = trained
    path = str(tmp_path / "filter.npz")
    sur.save(path)
    back = PF.Surrogate.load(path)
    assert back.fingerprint() == sur.fingerprint()
    lib = P.DeviceLibrary(I.make_ligands(500, W.dist, W.n_types, stream="sample"))
    say("saved and reloaded filter: predictions of 500 ligands")
    assert np.array_equal(back.predict_library(lib), sur.predict_library(lib))
    assert back.metrics["best_epochs"] == sur.metrics["best_epochs"]
