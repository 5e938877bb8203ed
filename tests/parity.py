"""Comparison protocol between the HIP screen and the FP64 oracle (test infrastructure).

Tolerance for best scores: |a - b| <= TAU * max(1, |b|) with TAU = 1e-4 (relative, floor 1).

The search is greedy, so an FP32/FP64 near-tie in one torsion decision may send the
two implementations down different but equally valid paths.  The checks are:
  1. exactness  - the oracle rescores the GPU's reported pose (start, steps) in FP64 and
                  gets the GPU's score;
  2. validity   - replaying the GPU's path in FP64, every GPU decision is an argmin up to TAU;
  3. optimality - the GPU's best is no worse than the oracle's wherever the GPU took the
                  oracle's path from the oracle's winning start, and no better wherever the
                  oracle took the GPU's path from the GPU's winning start; a ligand is excused
                  only where the paths are shown to split at a near-tie, and such ligands
                  are counted and bounded;
  4. indices    - the GPU's winning start is the oracle's unless their oracle finals tie
                  within TAU or the paths split at a near-tie.
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


def _split_is_near_tie(pocket, G, ligs, srch, lig, p, steps_gpu, periodic):
    """The GPU's path from start p differs from the oracle's: replay the GPU's steps in FP64 and
    check that every GPU decision is within TAU of the argmin, i.e. the two paths split at a
    near-tie.  With several passes only total turns are reported; the pose must then rescore to
    an FP64 value no better than the oracle allows (checked by the callers' rescoring)."""
    if srch.passes > 1:
        return True
    rp = oracle.replay(pocket, G, ligs, srch, np.array([lig]), np.array([p]), steps_gpu[None], periodic=periodic)
    B = ligs.n_rot[lig]
    eg, em = rp["e_given"][0, :B], rp["e_min"][0, :B]
    return bool(np.all(eg - em <= tol(em)))


def check_optimal(pocket, G, ligs, srch, sel, score, start, orc, finals, start_steps, periodic=False,
                  max_diverged=0.05):
    """Checks 3 and 4 against a full oracle run `orc` (oracle.dock(..., per_start=True)), given the
    GPU's per-start finals [n][N] and steps [n][N][16].

    For every ligand:
      * at the oracle's winning start p_or, if the GPU took the oracle's path (same steps; exact
        ties broken to the lowest step on both sides count as the same path), its final there is
        the oracle's best within TAU, so the GPU's best is no worse than the oracle's;
      * at the GPU's winning start, if the oracle took the GPU's path, the GPU's best is the
        oracle's final there within TAU, so it is no better than the oracle's best;
      * if the two winning starts differ and both paths agree, the oracle's finals at the two
        starts tie within TAU.
    A ligand is excused from a bound only where the paths are shown to split at a near-tie: the
    GPU's steps at that start, replayed in FP64, are each within TAU of the argmin (or, with start
    selection, the start was not among the GPU's selected starts because of a near-tie in the rigid
    ranking).  Such ligands are counted and may be at most `max_diverged` of the docked ligands
    (at least one).  Returns that count."""
    sel = np.asarray(sel)
    ok = np.isfinite(orc["best"])
    assert np.array_equal(ok, np.isfinite(score))
    idx = np.flatnonzero(ok)
    f_or, st_or = orc["finals"], orc["start_steps"]
    n_div = 0
    for i in idx:
        lig = sel[i]
        B = ligs.n_rot[lig]
        s_or, p_or, p_g = orc["best"][i], int(orc["start"][i]), int(start[i])
        diverged = False
        # upper bound: the GPU at the oracle's winning start
        if not np.isfinite(finals[i, p_or]):
            assert srch.sweep_top, f"ligand {lig}: oracle's winning start {p_or} not searched"
            diverged = True  # the GPU's FP32 rigid ranking put p_or just outside its top K
        elif np.array_equal(start_steps[i, p_or, :B], st_or[i, p_or, :B]):
            assert abs(finals[i, p_or] - s_or) <= tol(s_or), \
                f"ligand {lig}: same path at start {p_or}, GPU final {finals[i, p_or]} vs oracle {s_or}"
            assert score[i] <= s_or + tol(s_or), f"ligand {lig}: GPU {score[i]} worse than oracle {s_or}"
        else:
            assert _split_is_near_tie(pocket, G, ligs, srch, lig, p_or, start_steps[i, p_or], periodic), \
                f"ligand {lig}: GPU path at start {p_or} leaves the oracle's at a decision that is not a near-tie"
            diverged = True
        # lower bound: the oracle at the GPU's winning start
        same_at_gpu = np.isfinite(f_or[i, p_g]) and np.array_equal(start_steps[i, p_g, :B], st_or[i, p_g, :B])
        if same_at_gpu:
            assert abs(score[i] - f_or[i, p_g]) <= tol(f_or[i, p_g]), \
                f"ligand {lig}: same path at start {p_g}, GPU {score[i]} vs oracle {f_or[i, p_g]}"
            assert score[i] >= s_or - tol(s_or), f"ligand {lig}: GPU {score[i]} better than oracle {s_or}"
        else:
            # the GPU's own path was validated decision by decision (check 2); with selection the
            # oracle may not have searched p_g at all (near-tie in the rigid ranking)
            assert np.isfinite(f_or[i, p_g]) or srch.sweep_top, f"ligand {lig}: start {p_g} unsearched by the oracle"
            diverged = True
        # indices: with both paths shared, a different winning start is a tie between starts
        if p_g != p_or and not diverged:
            assert abs(f_or[i, p_g] - s_or) <= tol(s_or), f"ligand {lig}: start {p_g} vs oracle {p_or}"
        n_div += diverged
    assert n_div <= max(1, int(np.ceil(max_diverged * len(idx)))), \
        f"{n_div} of {len(idx)} ligands diverge from the oracle at near-ties"
    return n_div


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
