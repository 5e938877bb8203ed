"""Parity of the HIP screen with the oracle on random ligands drawn by Hypothesis (derandomized, so every
run draws the same examples): batches of trees of up to 40 atoms, degree <= 4, random rotatable bonds
and atom types, screened through the C ABI with 8, 64 or 100 torsion steps (one angle group per lane,
idle lanes, a ragged second group), against the oracle's statuses, its FP64 rescoring of every reported
pose, and its best poses."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from parity import check_exact_and_valid, check_optimal
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
