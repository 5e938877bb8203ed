"""Comparison protocol between the HIP screen and the FP64 oracle (test infrastructure).

Tolerance for best scores: |a - b| <= TAU * max(1, |b|) with TAU = 1e-4 (relative, floor 1).

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
# Arbitrary (unphysical) poses and the finals of non-winning starts can put atoms on the steep walls
# next to the +10 cap.  There the FP32 rounding of a position (a few ulp of the coordinate, in grid
# units) times the wall slope costs far more than TAU.  Such comparisons use TAU plus a per-atom
# allowance, PER_ATOM, that covers typical rounding, and they must all stay within the bound
# derived from the grid: TAU + sqrt(n) * slope * 4 ulp(coordinate), with slope the largest
# difference between neighbouring grid nodes.  A wrong term costs O(0.1-10) and fails both.
PER_ATOM = 2e-5


def tol(ref):
    return TAU * np.maximum(1.0, np.abs(ref))


def tol_pose(ref, n_atoms):
    return tol(ref) + PER_ATOM * np.asarray(n_atoms)


def grid_slope(G) -> float:
    """Largest change of a grid value between neighbouring nodes (per grid unit)."""
    return float(max(np.abs(np.diff(G, axis=a)).max() for a in (1, 2, 3)))


def tol_fp32(ref, n_atoms, G, dims):
    ulp = np.spacing(np.float32(max(dims)))  # coordinates in grid units stay below max(dims)
    return tol(ref) + np.sqrt(np.asarray(n_atoms, dtype=np.float64)) * grid_slope(G) * 4 * float(ulp)


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
    if srch.passes > 1:  # only each torsion's total turn is reported: no single decisions to replay
        return float(np.max(err / np.maximum(1.0, np.abs(e64))))
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


def check_per_start(pocket, G, ligs, srch, finals_gpu, steps_gpu, orc, periodic=False):
    """Per-start finals.  A start either agrees with the oracle's final, or the GPU took another
    path from it (an FP32/FP64 near-tie in some decision): then that path, replayed in FP64, must be
    made of near-argmin decisions and rescore to the GPU's final.  Agreement is within tol_fp32 for
    every start and within tol_pose for all but a small fraction.  Returns counts."""
    sel = orc["sel"]
    f_or, gap = orc["finals"], orc["start_gap"]
    n_at = ligs.n_atoms[sel][:, None]
    ok = np.isfinite(f_or)
    assert np.array_equal(ok, np.isfinite(finals_gpu))
    bound = tol_fp32(f_or, n_at, G, pocket.dims)
    diff = np.abs(np.where(ok, finals_gpu, 0.0) - np.where(ok, f_or, 0.0))  # unsearched starts are +inf on both sides
    agree = ok & (diff <= bound)
    typical = ok & (diff <= tol_pose(f_or, n_at))
    div = np.argwhere(ok & ~agree)
    if len(div) and srch.passes > 1:
        # several passes report only each torsion's total turn: the GPU's pose must rescore to its
        # final in FP64 (the decisions themselves cannot be replayed)
        li, pi = div[:, 0], div[:, 1]
        e64 = oracle.score_poses(pocket, G, ligs, srch, sel[li], pi, steps_gpu[li, pi], periodic=periodic)
        lim = tol_fp32(e64, ligs.n_atoms[sel[li]], G, pocket.dims)
        assert np.all(np.abs(e64 - finals_gpu[li, pi]) <= lim), "a diverged multi-pass start does not rescore"
    elif len(div):
        li, pi = div[:, 0], div[:, 1]
        rp = oracle.replay(pocket, G, ligs, srch, sel[li], pi, steps_gpu[li, pi], periodic=periodic)
        B = ligs.n_rot[sel[li]]
        n_l = ligs.n_atoms[sel[li]]
        for r in range(len(div)):
            eg, em = rp["e_given"][r, :B[r]], rp["e_min"][r, :B[r]]
            lim = tol_fp32(em, n_l[r], G, pocket.dims)
            assert np.all(eg - em <= lim), f"start {div[r].tolist()}: GPU decision not a near-argmin ({eg - em})"
            assert abs(rp["final"][r] - finals_gpu[li[r], pi[r]]) <= tol_fp32(rp["final"][r], n_l[r], G, pocket.dims), \
                (f"start {div[r].tolist()}: GPU final {finals_gpu[li[r], pi[r]]!r}, FP64 of the GPU path "
                 f"{rp['final'][r]!r}, oracle final {f_or[li[r], pi[r]]!r}, steps {steps_gpu[li[r], pi[r], :B[r]]}, "
                 f"e_given {eg}, e_min {em}")
    err = diff / np.maximum(1.0, np.abs(np.where(ok, f_or, 0.0)))
    return {"starts": int(ok.sum()), "agree": int(agree.sum()), "agree_typical": int(typical.sum()),
            "diverged_valid": int(len(div)), "near_tie_starts": int((ok & (gap < TAU)).sum()),
            "max_rel_err_agree": float(err[agree].max(initial=0.0)), "slope": grid_slope(G)}
