"""Comparison protocol between the HIP screen and the FP64 oracle (test infrastructure).

Tolerance: |a - b| <= TAU * max(1, |b|) with TAU = 1e-4 (relative, floor 1).

The search is greedy, so an FP32/FP64 near-tie in one torsion decision may send the
two implementations down different but equally valid paths.  The checks are:
  1. exactness  - the oracle rescores the GPU's reported pose (start, steps) in FP64 and
                  gets the GPU's score;
  2. validity   - replaying the GPU's path in FP64, every GPU decision is an argmin up to TAU;
  3. optimality - the GPU's best is no worse than the oracle's when the oracle's winning
                  path has no near-tie, and no better when the oracle's own path from the
                  GPU's winning start has no near-tie;
  4. indices    - the GPU's winning start is the oracle's unless their oracle finals tie
                  within TAU or a near-tie was met.
"""
import numpy as np

import oracle

TAU = 1e-4
# Arbitrary (unphysical) poses put atoms on the steep walls next to the +10 cap, where FP32
# rounding of a position (a few ulp of ~16 A, i.e. ~1e-5 A after the torsion moves, ~3e-5 grid
# units) times a wall slope of up to ~25 per grid unit gives up to ~7e-4 per atom in the worst
# cell.  Such poses are compared with TAU plus 2e-5 per atom: well below that worst case (errors of
# different atoms do not add up coherently) and far below any wrong term, which is O(0.1-10).
# Best poses sit in smooth regions and are held to TAU alone.
PER_ATOM = 2e-5


def tol(ref):
    return TAU * np.maximum(1.0, np.abs(ref))


def tol_pose(ref, n_atoms):
    return tol(ref) + PER_ATOM * np.asarray(n_atoms)


def check_exact_and_valid(pocket, G, ligs, srch, sel, score, start, steps, periodic=False):
    """Checks 1 and 2 for the ligands `sel`; returns the max relative rescoring error."""
    sel = np.asarray(sel)
    ok = np.isfinite(score)
    assert np.all(start[~ok] == -1)
    if not ok.any():
        return 0.0
    s_ok, st_ok, sc_ok = sel[ok], start[ok], steps[ok]
    e64 = oracle.score_poses(pocket, G, ligs, srch, s_ok, st_ok, sc_ok, periodic=periodic)
    err = np.abs(score[ok] - e64)
    assert np.all(err <= tol(e64)), f"rescoring mismatch: max {np.max(err / np.maximum(1, np.abs(e64)))}"
    rp = oracle.replay(pocket, G, ligs, srch, s_ok, st_ok, sc_ok, periodic=periodic)
    B = ligs.n_rot[s_ok]
    for i in range(len(s_ok)):
        eg, em = rp["e_given"][i, :B[i]], rp["e_min"][i, :B[i]]
        assert np.all(eg - em <= tol(em)), f"ligand {s_ok[i]}: a GPU decision is not an argmin ({eg - em})"
    return float(np.max(err / np.maximum(1.0, np.abs(e64))))


def check_optimal(pocket, G, ligs, srch, sel, score, start, orc, periodic=False):
    """Checks 3 and 4 against a full oracle run `orc` (oracle.dock(..., per_start=True))."""
    sel = np.asarray(sel)
    n_flag = 0
    ok = np.isfinite(orc["best"])
    assert np.array_equal(ok, np.isfinite(score))
    idx = np.flatnonzero(ok)
    g_start = oracle.greedy_starts(pocket, G, ligs, srch, sel[idx], start[idx], periodic=periodic)
    for n, i in enumerate(idx):
        s_or, p_or = orc["best"][i], orc["start"][i]
        gap_or = orc["start_gap"][i, p_or]
        f_or_at_gpu, gap_at_gpu = g_start["final"][n], g_start["gap"][n]
        clean = gap_or >= TAU and gap_at_gpu >= TAU
        if gap_or >= TAU:
            assert score[i] <= s_or + tol(s_or), f"ligand {sel[i]}: GPU {score[i]} worse than oracle {s_or}"
        if gap_at_gpu >= TAU:
            assert score[i] >= s_or - tol(s_or), f"ligand {sel[i]}: GPU {score[i]} better than oracle {s_or}"
            assert abs(score[i] - f_or_at_gpu) <= tol(f_or_at_gpu)
        if start[i] != p_or:
            assert abs(f_or_at_gpu - s_or) <= tol(s_or) or not clean, \
                f"ligand {sel[i]}: start {start[i]} vs oracle {p_or}"
        n_flag += not clean
    return n_flag


def check_per_start(finals_gpu, orc, n_atoms):
    """Per-start finals: equal within TAU wherever the oracle's path from that start has no near-tie.
    Near-tie starts (a decision gap below TAU on the oracle's path, most often an exact tie of
    moving atoms that sit in cells at the cap) may legitimately differ and are only counted."""
    f_or, gap = orc["finals"], orc["start_gap"]
    clean = np.isfinite(f_or) & (gap >= TAU)
    err = np.abs(finals_gpu - f_or) / np.maximum(1.0, np.abs(f_or))
    bad = clean & (np.abs(finals_gpu - f_or) > tol_pose(f_or, n_atoms[:, None]))
    assert not bad.any(), f"{bad.sum()} starts differ; first {np.argwhere(bad)[:5].tolist()}"
    tie = ~clean & np.isfinite(f_or)
    tie_agree = tie & (np.abs(finals_gpu - f_or) <= tol_pose(f_or, n_atoms[:, None]))
    return {"compared": int(clean.sum()), "near_tie": int(tie.sum()), "near_tie_agree": int(tie_agree.sum()),
            "max_rel_err": float(err[clean].max(initial=0.0))}
