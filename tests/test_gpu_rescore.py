"""Pose filtering and rescoring on the GPU (dock_rescore) against the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _check_against_oracle(pocket, ligs, srch, fin, res, n_keep, rmsd_min):
    """Every ligand's picks, replayed poses, FP64 rescores, filter decisions and best pose against the
    oracle; returns the number of ligands whose filter decisions differ at an RMSD within 1e-4 of the
    threshold (FP32 poses)."""
    from paper_2304_09953_amd import pipeline as P
    n, QT = fin.shape
    start = res.pose_start.cpu().numpy()
    steps = P.steps_numpy(res.pose_steps.view(-1)).reshape(n, n_keep, -1)
    score = res.pose_score.cpu().numpy()
    resc = res.pose_rescore.cpu().numpy().astype(np.float64)
    xyz = res.pose_xyz.cpu().numpy()
    best, best_pose = res.best_rescore.cpu().numpy(), res.best_pose.cpu().numpy()
    flips = 0
    for l in range(n):
        # picks: the n_keep lowest finals of this screen (the same FP32 values), ties to the lower start
        order = np.lexsort((np.arange(QT), fin[l]))[:n_keep]
        order = order[np.isfinite(fin[l][order])]
        want = np.full(n_keep, -1)
        want[:len(order)] = order
        assert np.array_equal(start[l], want), l
        live = start[l] >= 0
        assert np.array_equal(score[l][live], fin[l][start[l][live]])  # the replay reproduces the screen
        orc = oracle.filter_rescore(pocket, ligs, srch, l, start[l], steps[l], rmsd_min)
        kept = np.isfinite(resc[l])
        na = ligs.n_atoms[l]
        for i in np.flatnonzero(kept):
            X = oracle.pose_coords(ligs, srch, l, int(start[l][i]), steps[l][i])
            assert np.abs(xyz[l, i, :na] - X).max() < 1e-4  # the FP32 pose against the FP64 one
            ref = oracle.rescore_conformer(pocket, ligs, srch, l, xyz[l, i, :na])
            assert abs(resc[l][i] - ref) <= 1e-6 * max(1.0, abs(ref)), (l, i, resc[l][i], ref)
        # filter decisions agree up to the first RMSD within 1e-4 of the threshold (FP32 poses)
        for i in range(n_keep):
            if kept[i] != orc["kept"][i]:
                assert abs(orc["nearest"][i] - rmsd_min) < 1e-4, (l, i, orc["nearest"][i])
                flips += 1
                break
        # best: the lowest kept rescore, ties to the earlier slot
        if kept.any():
            b = int(np.flatnonzero(kept)[np.argmin(resc[l][kept])])
            assert best_pose[l] == b and best[l] == np.float32(resc[l][b])
        else:
            assert best_pose[l] == -1 and np.isinf(best[l])
        if rmsd_min == 0.0:
            assert np.array_equal(kept, live)
    return flips


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket48-lib100")
    pocket = W.pockets[0]
    ligs = W.ligands().subset(np.arange(0, 100, 5))
    return P, W, pocket, ligs, P.DevicePocket(pocket), P.DeviceLibrary(ligs)


@pytest.mark.parametrize("n_keep,rmsd_min,top,passes,restarts",
                         [(8, 1.0, 0, 1, 0), (16, 2.5, 40, 2, 0), (3, 0.0, 0, 1, 0), (8, 1.0, 0, 1, 2)])
def test_rescore_matches_oracle(env, n_keep, rmsd_min, top, passes, restarts):
    P, W, pocket, ligs, dp, lib = env
    srch = dataclasses.replace(W.search, sweep_top=top, passes=passes, restarts=restarts,
                               init_steps=I.restart_steps(restarts, W.search.n_steps) if restarts else None)
    ds = P.DeviceSearch(srch)
    QT, n = srch.n_searched, ligs.n_lig  # searched starts: with restarts, (1 + R) rigid-start sets
    say(f"rescore: keep {n_keep}, rmsd_min {rmsd_min}, sweep_top {top}, passes {passes}, restarts {restarts}")
    scr = P.screen(dp, lib, ds, start_scores=True)
    res = P.rescore(dp, lib, ds, scr.start_scores.view(n, QT), n_keep, rmsd_min, want_xyz=True)
    torch.cuda.synchronize()
    fin = scr.start_scores.view(n, QT).cpu().numpy()
    flips = _check_against_oracle(pocket, ligs, srch, fin, res, n_keep, rmsd_min)
    say(f"threshold flips: {flips}")
    assert flips <= 1


@pytest.mark.timeout(600)
def test_rescore_at_full_size():
    """The benchmark's pocket and search (96^3 x 16 types, 256 quaternions x 32 translations, S = 256) on
    a stratified handful of its library: the largest and the smallest ligand, one with 12 torsions, one
    with none, and four seeded draws; 8 poses kept per ligand, 1 A apart."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    lib_all = W.ligands(n_lig=3000)
    n_rot = lib_all.n_rot
    pick = [int(np.argmax(lib_all.n_atoms)), int(np.argmin(lib_all.n_atoms)), int(np.flatnonzero(n_rot == 12)[0]),
            int(np.flatnonzero(n_rot == 0)[0])]
    rest = np.setdiff1d(np.arange(lib_all.n_lig), pick)
    pick += np.random.default_rng(3).choice(rest, 4, replace=False).tolist()
    sel = np.sort(np.unique(pick))
    ligs = lib_all.subset(sel)
    say(f"rescore at full size: ligands {sel.tolist()} (n {ligs.n_atoms.tolist()}, B {ligs.n_rot.tolist()}), "
        "keep 8, rmsd_min 1.0")
    dp, lib, ds = P.DevicePocket(pocket), P.DeviceLibrary(ligs), P.DeviceSearch(W.search)
    n, QT = ligs.n_lig, W.search.n_searched
    scr = P.screen(dp, lib, ds, start_scores=True)
    res = P.rescore(dp, lib, ds, scr.start_scores.view(n, QT), 8, 1.0, want_xyz=True)
    torch.cuda.synchronize()
    fin = scr.start_scores.view(n, QT).cpu().numpy()
    flips = _check_against_oracle(pocket, ligs, W.search, fin, res, 8, 1.0)
    say(f"full size: threshold flips {flips}, kept poses {np.isfinite(res.pose_rescore.cpu().numpy()).sum(1).tolist()}")
    assert flips <= 1


def test_rescore_is_layout_independent(env):
    # the pose replay runs the screen's lookups, which give the same values in both grid layouts
    P, W, pocket, ligs, _, lib = env
    ds = P.DeviceSearch(W.search)
    n, QT = ligs.n_lig, W.search.n_searched
    outs = []
    for layout in (0, 1):
        say(f"rescore: keep 8, rmsd_min 1.0, layout {layout}")
        dp = P.DevicePocket(pocket, layout=layout)
        scr = P.screen(dp, lib, ds, start_scores=True)
        res = P.rescore(dp, lib, ds, scr.start_scores.view(n, QT), 8, 1.0, want_xyz=True)
        torch.cuda.synchronize()
        outs.append({k: getattr(res, k).cpu() for k in ("pose_start", "pose_steps", "pose_score", "pose_rescore",
                                                         "pose_xyz", "best_rescore", "best_pose")})
    for k in outs[0]:
        assert torch.equal(outs[0][k], outs[1][k]) or (
            outs[0][k].dtype.is_floating_point and torch.equal(outs[0][k].nan_to_num(7.0), outs[1][k].nan_to_num(7.0))), k


def test_refused_rescore_enqueues_nothing(env):
    """A negative well depth is an argument error: the call returns it before any launch, so the
    outputs keep what they held."""
    P, W, pocket, ligs, dp, lib = env
    from paper_2304_09953_amd import dock
    ds = P.DeviceSearch(W.search)
    n, QT = ligs.n_lig, W.search.n_searched
    say("rescore with a negative eps is refused before any launch")
    scr = P.screen(dp, lib, ds, start_scores=True)
    dev = dp.grids.device
    sentinel = [torch.full((n, 4), -7, dtype=torch.int32, device=dev),
                torch.full((n, 4, dock.MAX_TORSIONS), -7, dtype=torch.int16, device=dev),
                torch.full((n, 4), -7.0, device=dev), torch.full((n, 4), -7.0, device=dev),
                torch.full((n,), -7.0, device=dev), torch.full((n,), -7, dtype=torch.int32, device=dev)]
    before = [t.clone() for t in sentinel]
    pk = pocket
    eps = np.array(pk.type_eps, dtype=np.float64).copy()
    eps[-1] = -0.1
    with pytest.raises(dock.DockError):
        dock.rescore(dp.desc, dp.grids, lib.pack, n, lib.n_atoms, ds.desc, scr.start_scores.view(n, QT), dp.prot_xyz,
                     dp.prot_type, pk.type_R, eps, pk.type_q, pk.cap, pk.r_min, pk.coulomb_k, 4, 1.0, *sentinel)
    torch.cuda.synchronize()
    for a, b in zip(sentinel, before):
        assert torch.equal(a, b)
