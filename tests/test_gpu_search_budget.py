"""Search-budget variants on the GPU against the oracle: torsion sweeps from only the K best
rigid starts, several greedy passes over the torsions, and torsion restarts of every rigid start."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from parity import check_exact_and_valid, check_optimal, check_per_start, tol_fp32
from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket48-lib100")
    pocket = W.pockets[0]
    ligs = W.ligands().subset(np.arange(0, 100, 5))
    return P, W, pocket, oracle.build_grids(pocket), ligs, P.DevicePocket(pocket)


def _screen(P, dp, ligs, srch):
    lib = P.DeviceLibrary(ligs)
    r = P.screen(dp, lib, P.DeviceSearch(srch), start_scores=True)
    torch.cuda.synchronize()
    n = ligs.n_lig
    return {"score": r.best_score.cpu().numpy().astype(np.float64), "start": r.best_start.cpu().numpy(),
            "steps": P.steps_numpy(r.best_steps), "poses": int(r.pose_count.cpu().item()),
            "finals": r.start_scores.cpu().numpy().reshape(n, -1).astype(np.float64),
            "start_steps": P.steps_numpy(r.start_steps).reshape(n, srch.n_searched, -1)}


@pytest.mark.parametrize("top,passes", [(16, 1), (0, 2), (40, 3)])
def test_search_budget_matches_oracle(env, top, passes):
    P, W, pocket, G, ligs, dp = env
    srch = dataclasses.replace(W.search, sweep_top=top, passes=passes)
    QT = srch.n_starts
    say(f"pocket48-lib100 subset of 20: sweep_top={top}, passes={passes}")
    g = _screen(P, dp, ligs, srch)
    every = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, sweep_top=0), per_start=True)
    searched = np.isfinite(g["finals"])
    n_searched = top if top else QT
    assert np.all(searched.sum(1) == n_searched)
    if top:
        # the searched starts are the K lowest rigid scores, up to FP32 rounding of those scores
        for l in range(ligs.n_lig):
            rig = oracle.score_poses(pocket, G, ligs, srch, np.full(QT, l), np.arange(QT), np.zeros((QT, 16), int))
            lim = tol_fp32(rig, ligs.n_atoms[l], G, pocket.dims).max()
            assert rig[searched[l]].max() <= rig[~searched[l]].min() + 2 * lim
    # per-start finals of the searched starts against the oracle's greedy from the same starts
    orc = dict(every)
    orc["finals"] = np.where(searched, every["finals"], np.inf)
    st = check_per_start(pocket, G, ligs, srch, g["finals"], g["start_steps"], orc)
    say(f"per-start: {st}")
    assert st["agree"] >= 0.99 * st["starts"]
    assert np.array_equal(g["score"], g["finals"].min(1))
    assert np.array_equal(g["start"], np.argmin(g["finals"], 1))
    sel = np.arange(ligs.n_lig)
    check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
    # the best over the GPU's searched starts against the oracle's best over the same starts
    f = orc["finals"]
    orc["best"] = f.min(1)
    orc["start"] = np.argmin(f, 1).astype(np.int32)
    n_flag = check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    say(f"{n_flag} ligands whose paths split from the oracle's at near-ties")
    B = ligs.n_rot
    assert g["poses"] == int(np.sum(QT + n_searched * passes * B * (srch.n_steps - 1)))


def test_selecting_every_start_is_the_plain_search(env):
    P, W, pocket, G, ligs, dp = env
    say("sweep_top = Q*T and = Q*T + 7 against sweep_top = 0")
    base = _screen(P, dp, ligs, W.search)
    for K in (W.search.n_starts, W.search.n_starts + 7):
        r = _screen(P, dp, ligs, dataclasses.replace(W.search, sweep_top=K))
        for key in ("score", "start", "steps", "finals", "start_steps", "poses"):
            assert np.array_equal(np.asarray(r[key]), np.asarray(base[key])), key


@pytest.mark.parametrize("restarts,passes", [(2, 1), (3, 2)])
def test_restarts_match_oracle(env, restarts, passes):
    P, W, pocket, G, ligs, dp = env
    srch = dataclasses.replace(W.search, passes=passes, restarts=restarts,
                               init_steps=I.restart_steps(restarts, W.search.n_steps))
    N, QT = srch.n_searched, srch.n_starts
    say(f"pocket48-lib100 subset of 20: {restarts} torsion restarts per start, passes={passes}")
    g = _screen(P, dp, ligs, srch)
    orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
    assert g["finals"].shape == (ligs.n_lig, N) and np.all(np.isfinite(g["finals"]))
    st = check_per_start(pocket, G, ligs, srch, g["finals"], g["start_steps"], orc)
    say(f"per-start: {st}")
    assert st["agree"] >= 0.99 * st["starts"]
    assert np.array_equal(g["score"], g["finals"].min(1)) and np.array_equal(g["start"], np.argmin(g["finals"], 1))
    sel = np.arange(ligs.n_lig)
    check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
    n_flag = check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    say(f"{n_flag} ligands split at near-ties; restart winners: {int(np.sum(g['start'] >= QT))} of {ligs.n_lig}")
    B = ligs.n_rot
    assert g["poses"] == int(np.sum(N * (1 + passes * B * (srch.n_steps - 1))))


@pytest.mark.timeout(600)
def test_restarts_and_passes_at_full_size():
    """The benchmark's pocket and search (96^3 x 16 types, 256 x 32 rigid starts, S = 256) with one torsion
    restart of every rigid start and two greedy passes (16384 searched starts per ligand), on two of its
    ligands of median size, against the oracle start by start."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    lib_all = W.ligands(n_lig=400)
    med = np.flatnonzero((np.abs(lib_all.n_atoms - 30) <= 3) & (lib_all.n_rot >= 3) & (lib_all.n_rot <= 5))[:2]
    ligs = lib_all.subset(med)
    srch = dataclasses.replace(W.search, passes=2, restarts=1, init_steps=I.restart_steps(1, W.search.n_steps))
    N, QT = srch.n_searched, srch.n_starts
    say(f"pocket96 full size, ligands {med.tolist()} (n {ligs.n_atoms.tolist()}, B {ligs.n_rot.tolist()}): "
        f"1 restart per start, 2 passes, {N} searched starts each")
    G = oracle.build_grids(pocket)
    g = _screen(P, P.DevicePocket(pocket), ligs, srch)
    orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
    assert g["finals"].shape == (ligs.n_lig, N) and np.all(np.isfinite(g["finals"]))
    st = check_per_start(pocket, G, ligs, srch, g["finals"], g["start_steps"], orc)
    say(f"per-start: {st}")
    assert st["agree"] >= 0.99 * st["starts"]
    assert np.array_equal(g["score"], g["finals"].min(1)) and np.array_equal(g["start"], np.argmin(g["finals"], 1))
    sel = np.arange(ligs.n_lig)
    check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
    n_flag = check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    say(f"{n_flag} ligands split at near-ties; best {g['score'].tolist()} vs oracle {orc['best'].tolist()}")
    assert g["poses"] == int(np.sum(N * (1 + 2 * ligs.n_rot * (srch.n_steps - 1))))


def test_zero_restarts_repeat_the_plain_search(env):
    P, W, pocket, G, ligs, dp = env
    say("two restarts with zero initial turns against the plain search")
    base = _screen(P, dp, ligs, W.search)
    r = _screen(P, dp, ligs, dataclasses.replace(W.search, restarts=2, init_steps=np.zeros((2, 16), np.int32)))
    QT = W.search.n_starts
    for k in range(3):
        assert np.array_equal(r["finals"][:, k * QT:(k + 1) * QT], base["finals"])
        assert np.array_equal(r["start_steps"][:, k * QT:(k + 1) * QT], base["start_steps"])
    for key in ("score", "start", "steps"):
        assert np.array_equal(np.asarray(r[key]), np.asarray(base[key])), key


@pytest.mark.parametrize("boundary", [0, 1])
def test_budget_variants_are_layout_independent(env, boundary):
    # selection, passes and restarts run through the same lookups in both grid layouts, so the two
    # give the same screen bit for bit, under either boundary mode
    P, W, pocket, G, ligs, _ = env
    variants = [dict(sweep_top=16, passes=2), dict(restarts=2, init_steps=I.restart_steps(2, W.search.n_steps))]
    for v in variants:
        srch = dataclasses.replace(W.search, **v)
        runs = []
        for layout in (0, 1):
            say(f"pocket48-lib100 subset of 20: {sorted(v)}, boundary {boundary}, layout {layout}")
            runs.append(_screen(P, P.DevicePocket(pocket, boundary=boundary, layout=layout), ligs, srch))
        for key in ("score", "start", "steps", "poses", "finals", "start_steps"):
            assert np.array_equal(runs[0][key], runs[1][key]), (v, key)
