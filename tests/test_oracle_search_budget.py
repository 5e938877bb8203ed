"""Pins of the oracle's search-budget variants: torsion sweeps from only the K best rigid starts,
several greedy passes over the torsions, and torsion restarts of every rigid start."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2304_09953_amd import inputs as I


@pytest.fixture(scope="module")
def case():
    pocket = I.make_pocket(40, 4, pocket_id=21)
    G = oracle.build_grids(pocket)
    ligs = I.make_ligands(6, I.DIST_DRUGLIKE, 4, stream="test", first_id=500)
    srch = I.make_search(6, 4, 24, 3.0, pocket.center)
    base = oracle.dock(pocket, G, ligs, srch, per_start=True)
    return pocket, G, ligs, srch, base


def _rigid(pocket, G, ligs, srch, l):
    QT = srch.n_starts
    return oracle.score_poses(pocket, G, ligs, srch, np.full(QT, l), np.arange(QT), np.zeros((QT, 16), int))


def test_all_starts_selected_is_the_plain_search(case):
    pocket, G, ligs, srch, base = case
    for K in (0, srch.n_starts, srch.n_starts + 5):
        r = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, sweep_top=K), per_start=True)
        assert np.array_equal(r["finals"], base["finals"]) and np.array_equal(r["start"], base["start"])


@pytest.mark.parametrize("K", [1, 5])
def test_top_k_searches_the_k_best_rigid_starts(case, K):
    pocket, G, ligs, srch, base = case
    r = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, sweep_top=K), per_start=True)
    for l in range(ligs.n_lig):
        rig = _rigid(pocket, G, ligs, srch, l)
        chosen = np.lexsort((np.arange(srch.n_starts), rig))[:K]
        searched = np.flatnonzero(np.isfinite(r["finals"][l]))
        assert np.array_equal(np.sort(chosen), searched)
        # the searched starts' greedy results are those of the plain search
        assert np.array_equal(r["finals"][l][searched], base["finals"][l][searched])
        assert np.array_equal(r["start_steps"][l][searched], base["start_steps"][l][searched])
        b = np.lexsort((searched, base["finals"][l][searched]))[0]
        assert r["start"][l] == searched[b] and r["best"][l] == base["finals"][l][searched[b]]
        # sweeps never raise a start's score, so the best is at most the best rigid score
        assert r["best"][l] <= rig.min() + 1e-12


def test_second_pass_never_raises_a_score_and_totals_reproduce_the_pose(case):
    pocket, G, ligs, srch, base = case
    two = dataclasses.replace(srch, passes=2)
    r = oracle.dock(pocket, G, ligs, two, per_start=True)
    assert np.all(r["finals"] <= base["finals"] + 1e-12)
    nrot = ligs.n_rot
    for l in range(ligs.n_lig):
        if nrot[l] <= 1:  # one torsion: its first sweep already found the best of the circle
            assert np.array_equal(r["finals"][l], base["finals"][l])
    # torsion turns change only their own torsion angle: the reference conformer with each torsion
    # turned once by its total (the sum of its steps over the passes, mod S) is the final conformer
    QT = srch.n_starts
    for l in range(ligs.n_lig):
        p = np.arange(QT)
        sc = oracle.score_poses(pocket, G, ligs, two, np.full(QT, l), p, r["start_steps"][l])
        assert np.allclose(sc, r["finals"][l], rtol=1e-10, atol=1e-10)
    assert np.any(r["finals"] < base["finals"] - 1e-6)  # the second pass does improve some starts
    assert np.all(r["start_steps"] < srch.n_steps)


def test_zero_restarts_reproduce_the_rigid_starts(case):
    pocket, G, ligs, srch, base = case
    r = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, restarts=2, init_steps=np.zeros((2, 16), np.int32)),
                    per_start=True)
    QT = srch.n_starts
    for k in range(3):  # searched start k QT + p is restart k of rigid start p
        assert np.array_equal(r["finals"][:, k * QT:(k + 1) * QT], base["finals"])
        assert np.array_equal(r["start_steps"][:, k * QT:(k + 1) * QT], base["start_steps"])
    assert np.array_equal(r["best"], base["best"]) and np.array_equal(r["start"], base["start"])


def test_restart_from_a_final_pose_never_gets_worse(case):
    # a restart whose initial turns are a start's final totals begins at that final pose; every sweep
    # offers step 0, so its own final is no worse
    pocket, G, ligs, srch, base = case
    QT = srch.n_starts
    for l in range(ligs.n_lig):
        p = int(base["start"][l])
        init = base["start_steps"][l, p][None].astype(np.int32)
        r = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, restarts=1, init_steps=init), sel=[l],
                        per_start=True)
        assert r["finals"][0, QT + p] <= base["best"][l] + 1e-12 * max(1.0, abs(base["best"][l]))
        assert r["best"][0] <= base["best"][l]


def test_restart_results_rescore_and_replay(case):
    pocket, G, ligs, srch, base = case
    R = 3
    rs = dataclasses.replace(srch, restarts=R, init_steps=I.restart_steps(R, srch.n_steps))
    r = oracle.dock(pocket, G, ligs, rs, per_start=True)
    N = rs.n_searched
    assert r["finals"].shape == (ligs.n_lig, N) and np.all(r["best"] <= base["best"])
    for l in range(ligs.n_lig):
        e = np.arange(N)
        # the reported steps are total turns from the rigid start e mod QT: rescoring them gives the final
        sc = oracle.score_poses(pocket, G, ligs, rs, np.full(N, l), e, r["start_steps"][l])
        assert np.allclose(sc, r["finals"][l], rtol=1e-12, atol=1e-12)
        rp = oracle.replay(pocket, G, ligs, rs, np.full(N, l), e, r["start_steps"][l])
        B = int(ligs.n_rot[l])
        assert np.array_equal(rp["e_given"][:, :B], rp["e_min"][:, :B])
        assert np.array_equal(rp["final"], r["finals"][l])
    # restarts are not combined with start selection
    with pytest.raises(ValueError):
        oracle.dock(pocket, G, ligs, dataclasses.replace(rs, sweep_top=4))
