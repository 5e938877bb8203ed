"""Parity of the HIP screen with the oracle on random ligands drawn by Hypothesis (derandomized, so every
run draws the same examples): batches of trees of up to 40 atoms, degree <= 4, random rotatable bonds
and atom types, screened through the C ABI with 8, 64 or 100 torsion steps (one angle group per lane,
idle lanes, a ragged second group), against the oracle's statuses, its FP64 rescoring of every reported
pose, and its best poses; and with the search-budget variants (start selection, several passes, torsion
restarts) start by start."""
import dataclasses

import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from parity import check_exact_and_valid, check_optimal, check_per_start
from paper_2304_09953_amd import inputs as I
from test_gpu_parity import _screen
from test_oracle_properties import trees

pytestmark = pytest.mark.gpu

N_TYPES = 8


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    pocket = I.make_pocket(40, N_TYPES, n_prot=200, pocket_id=31)
    say("40^3 pocket with 8 types for the random-ligand batches")
    return P, pocket, oracle.build_grids(pocket), P.DevicePocket(pocket)


@settings(max_examples=8, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(batch=st.lists(trees(max_n=40, n_types=N_TYPES), min_size=4, max_size=12), S=st.sampled_from([8, 64, 100]))
def test_random_ligands_match_the_oracle(env, batch, S):
    P, pocket, G, dp = env
    ligs = I.from_parts(batch, N_TYPES)
    srch = I.make_search(8, 2, S, 2.0, pocket.center)
    say(f"random batch of {ligs.n_lig} ligands (n {ligs.n_atoms.tolist()}, B {ligs.n_rot.tolist()}), S={S}")
    g = _screen(P, dp, ligs, srch, start_scores=True)
    status = oracle.status(ligs)
    assert np.array_equal(g["status"], status)
    assert np.all(status == 0)
    sel = np.arange(ligs.n_lig)
    check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
    orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
    n_div = check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    say(f"{n_div} ligands split from the oracle at near-ties")
    assert g["poses"] == oracle.pose_count(ligs.n_rot, status, srch.n_starts, S)


@st.composite
def budgets(draw):
    """(sweep_top, passes, restarts): restarts only with every start swept."""
    restarts = draw(st.sampled_from([0, 0, 1, 2]))
    top = 0 if restarts else draw(st.sampled_from([0, 3, 9]))
    return top, draw(st.integers(1, 2)), restarts


@settings(max_examples=6, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(batch=st.lists(trees(max_n=30, n_types=N_TYPES), min_size=3, max_size=8), S=st.sampled_from([16, 64]),
       budget=budgets())
def test_random_ligands_with_search_budgets_match_the_oracle(env, batch, S, budget):
    P, pocket, G, dp = env
    top, passes, restarts = budget
    ligs = I.from_parts(batch, N_TYPES)
    srch = dataclasses.replace(I.make_search(8, 2, S, 2.0, pocket.center), sweep_top=top, passes=passes,
                               restarts=restarts, init_steps=I.restart_steps(restarts, S) if restarts else None)
    say(f"random batch of {ligs.n_lig} ligands (n {ligs.n_atoms.tolist()}, B {ligs.n_rot.tolist()}), S={S}, "
        f"sweep_top {top}, passes {passes}, restarts {restarts}")
    lib = P.DeviceLibrary(ligs)
    r = P.screen(dp, lib, P.DeviceSearch(srch), start_scores=True)
    torch.cuda.synchronize()
    n, N = ligs.n_lig, srch.n_searched
    score, start = r.best_score.cpu().numpy().astype(np.float64), r.best_start.cpu().numpy()
    finals = r.start_scores.cpu().numpy().reshape(n, N).astype(np.float64)
    steps_all = P.steps_numpy(r.start_steps).reshape(n, N, -1)
    full = oracle.dock(pocket, G, ligs, dataclasses.replace(srch, sweep_top=0), per_start=True)
    searched = np.isfinite(finals)
    assert np.all(searched.sum(1) == (min(top, srch.n_starts) if top else N))
    orc = dict(full)
    orc["finals"] = np.where(searched, full["finals"], np.inf)
    stats = check_per_start(pocket, G, ligs, srch, finals, steps_all, orc)
    assert stats["agree"] >= 0.98 * stats["starts"], stats
    assert np.array_equal(score, finals.min(1)) and np.array_equal(start, np.argmin(finals, 1))
    sel = np.arange(n)
    check_exact_and_valid(pocket, G, ligs, srch, sel, score, start, P.steps_numpy(r.best_steps))
    orc["best"] = orc["finals"].min(1)
    orc["start"] = np.argmin(orc["finals"], 1).astype(np.int32)
    n_div = check_optimal(pocket, G, ligs, srch, sel, score, start, orc, finals, steps_all)
    say(f"per-start {stats}; {n_div} ligands split at near-ties")
