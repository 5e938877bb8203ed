"""Parity of the HIP docking path (through the C ABI) with the FP64 oracle.

Every case prints its name before touching the GPU so a failing run names it.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import TAU, check_exact_and_valid, check_optimal, check_per_start, tol, tol_fp32, tol_pose
from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import pipeline
    return pipeline


@pytest.fixture(scope="module")
def p48(P):
    W = I.workload("pocket48-lib100")
    pocket = W.pockets[0]
    say("48^3 pocket grids")
    dp = P.DevicePocket(pocket)
    return W, pocket, dp, oracle.build_grids(pocket), W.ligands()


# ------------------------------------------------------------------------------------------------
# Grids
# ------------------------------------------------------------------------------------------------

def test_grids_pocket48_match_oracle(p48):
    W, pocket, dp, G, _ = p48
    g = dp.view().cpu().numpy()
    err = np.abs(g.astype(np.float64) - G) / np.maximum(1.0, np.abs(G))
    say(f"48^3 grid max rel err {err.max():.3g}")
    assert err.max() <= 1e-6


def test_xy4_records_hold_the_wrapped_neighbours(P):
    pocket = I.make_pocket((40, 36, 28), 4, pocket_id=3)
    say("xy4 records vs the linear grid, 40x36x28 x 4")
    lin = P.DevicePocket(pocket, layout=0).view()
    rec = P.DevicePocket(pocket, layout=1).records()
    # dims of the [t][z][y][x] view: x is 3, y is 2
    lin_y = torch.roll(lin, -1, dims=2)
    d_x = torch.roll(lin, -1, dims=3) - lin  # FP32 differences
    assert torch.equal(rec[..., 0], lin)
    assert torch.equal(rec[..., 1], d_x)
    assert torch.equal(rec[..., 2], lin_y - lin)
    assert torch.equal(rec[..., 3], (torch.roll(lin_y, -1, dims=3) - lin_y) - d_x)
    # storage order: [t][z/2][y/2][x][z&1][y&1] records of 16 bytes
    dp = P.DevicePocket(pocket, layout=1)
    raw = dp.grids.view(4, 14, 18, 40, 2, 2, 4)
    # record (x 15, y 10, z 7): z/2 = 3, y/2 = 5, z&1 = 1, y&1 = 0
    g00, g10, g01, g11 = lin[1, 7, 10, 15], lin[1, 7, 10, 16], lin[1, 7, 11, 15], lin[1, 7, 11, 16]
    assert torch.equal(raw[1, 3, 5, 15, 1, 0], torch.stack([g00, g10 - g00, g01 - g00, (g11 - g01) - (g10 - g00)]))
    # odd dimensions: padding records are zero
    odd = I.make_pocket((13, 7, 5), 2, pocket_id=4)
    say("xy4 records of a 13x7x5 grid (padded to 14x8x6)")
    o_lin = P.DevicePocket(odd, layout=0).view()
    o_dp = P.DevicePocket(odd, layout=1)
    o_rec = o_dp.records()
    assert torch.equal(o_rec[..., 0], o_lin) and torch.equal(o_rec[..., 2], torch.roll(o_lin, -1, dims=2) - o_lin)
    assert o_dp.grids.numel() == 2 * 14 * 4 * 3 * 16
    full = o_dp.grids.view(2, 3, 4, 14, 2, 2, 4).permute(0, 1, 4, 2, 5, 3, 6).reshape(2, 6, 8, 14, 4)
    assert torch.all(full[:, 5:] == 0) and torch.all(full[:, :, 7:] == 0) and torch.all(full[:, :, :, 13:] == 0)
    back = P.DevicePocket(pocket, layout=1)
    back.grids.zero_()
    back.write_records(rec)
    assert torch.equal(back.grids, dp.grids)


def test_grids_96_sampled_nodes(P):
    pocket = I.make_pocket(96, 16)
    say("96^3 x 16 grid build")
    dp = P.DevicePocket(pocket)
    g = dp.view().cpu().numpy()
    rng = np.random.default_rng(7)
    tijk = np.stack([rng.integers(0, 16, 3000), rng.integers(0, 96, 3000), rng.integers(0, 96, 3000),
                     rng.integers(0, 96, 3000)], 1).astype(np.int32)
    ref = oracle.grid_nodes(pocket, tijk)
    got = g[tijk[:, 0], tijk[:, 3], tijk[:, 2], tijk[:, 1]].astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.maximum(1.0, np.abs(ref)))
    assert g.max() <= 10.0


# ------------------------------------------------------------------------------------------------
# Packer
# ------------------------------------------------------------------------------------------------

def _al(v):
    return (v + 255) & ~255


def decode_pack(pack: np.ndarray, n_lig: int, n_atoms: int):
    """Test-side reader of the packed library (layout of the internal pack format)."""
    o = 0
    desc_o = o; o = _al(o + 32 * n_lig)
    x_o = o; o = _al(o + 4 * n_atoms)
    y_o = o; o = _al(o + 4 * n_atoms)
    z_o = o; o = _al(o + 4 * n_atoms)
    t_o = o; o = _al(o + n_atoms)
    e_o = o; o = _al(o + 16 * n_atoms)
    tor_o = o
    desc = pack[desc_o:desc_o + 32 * n_lig].view(np.int32).reshape(n_lig, 8)
    xyz = np.stack([pack[a:a + 4 * n_atoms].view(np.float32) for a in (x_o, y_o, z_o)], 1)
    excl = pack[e_o:e_o + 16 * n_atoms].view(np.uint32).reshape(n_atoms, 4)
    tor = pack[tor_o:tor_o + 20 * 16 * n_lig].reshape(n_lig, 16, 20)
    return desc, xyz, excl, tor


def _mask_bits(words, n):
    return np.array([(words[i >> 5] >> (i & 31)) & 1 for i in range(n)], bool)


def _edge_library():
    from test_oracle_pins import chain
    parts = []
    for src, idx in ((I.make_ligands(30, I.DIST_HEAVY_TAIL, 16, stream="test"), range(30)),
                     (I.make_ligands(3, I.LibDist(fixed_n=128, fixed_b=16, b_max=16), 16, stream="test"), range(3)),
                     (I.make_ligands(3, I.LibDist(fixed_n=100, fixed_b=12), 16, stream="test"), range(3))):
        parts += [src.ligand(i) for i in idx]
    x, t, b, r = chain(5, [])
    parts += [
        (np.zeros((1, 3)), np.zeros(1, np.uint8), np.zeros((0, 2)), np.zeros(0, np.uint8)),  # single atom
        (np.array([[0, 0, 0], [1.5, 0, 0]]), np.zeros(2, np.uint8), [(0, 1)], [0]),          # two atoms, B = 0
        (x, np.array([0, 0, 17, 0, 0], np.uint8), b, r),                                      # bad type
        (x, t, b[:3], r[:3]),                                                                  # bad bond count
        (x, t, [(0, 1), (1, 2), (0, 1), (3, 4)], r),                                          # not a tree
        (x, t, b, [1, 0, 0, 0]),                                                               # terminal rotatable
        chain(129, []),                                                                        # too many atoms
        chain(20, [(i, i + 1) for i in range(1, 18)]),                                        # 17 torsions
        chain(19, [(i, i + 1) for i in range(1, 17)]),                                        # 16 torsions (max)
    ]
    return I.from_parts(parts, 16)


def test_pack_status_topology_and_centring(P):
    ligs = _edge_library()
    say(f"pack {ligs.n_lig} ligands incl. planted errors")
    lib = P.DeviceLibrary(ligs)
    torch.cuda.synchronize()
    st = lib.status.cpu().numpy()
    assert np.array_equal(st, oracle.status(ligs))
    assert set(st.tolist()) >= {0, 1, 2, 3, 6, 7, 8}
    desc, xyz, excl, tor = decode_pack(lib.pack.cpu().numpy(), ligs.n_lig, lib.n_atoms)
    for l in np.flatnonzero(st == 0):
        topo = oracle.topology(ligs, int(l))
        a0, n, B = desc[l, 0], desc[l, 1], desc[l, 2]
        assert n == ligs.n_atoms[l] and B == topo["B"]
        assert desc[l, 4] == topo["moving"].sum()
        assert desc[l, 5] == len(topo["pairs"])
        assert np.allclose(xyz[a0:a0 + n], topo["xref"], atol=2e-6, rtol=0)
        for k in range(B):
            rec = tor[l, k]
            words = rec[:16].view(np.uint32)
            assert (rec[16], rec[17]) == (topo["tor_a"][k], topo["tor_b"][k])
            assert np.array_equal(_mask_bits(words, n), topo["moving"][k])
            assert rec[18:20].view(np.uint16)[0] == topo["moving"][k].sum()
        pairs = set(map(tuple, topo["pairs"]))
        for i in range(n):
            ex = _mask_bits(excl[a0 + i], n)
            for j in range(n):
                assert ex[j] == ((min(i, j), max(i, j)) not in pairs)


# ------------------------------------------------------------------------------------------------
# Pose scoring
# ------------------------------------------------------------------------------------------------

def test_score_poses_vs_oracle(P, p48):
    W, pocket, dp, G, ligs = p48
    rng = np.random.default_rng(3)
    n = 3000
    lig = rng.integers(0, ligs.n_lig, n)
    start = rng.integers(0, W.search.n_starts, n)
    steps = rng.integers(0, W.search.n_steps, (n, 4))
    say("score_poses pocket48-lib100, 3000 random poses")
    lib = P.DeviceLibrary(ligs)
    ds = P.DeviceSearch(W.search)
    got = P.score_poses(dp, lib, ds, lig, start, steps).cpu().numpy()
    ref = oracle.score_poses(pocket, G, ligs, W.search, lig, start, steps)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    say(f"score_poses max rel err {err.max():.3g}, median {np.median(err):.3g}")
    assert np.all(np.abs(got - ref) <= tol_fp32(ref, ligs.n_atoms[lig], G, pocket.dims))
    assert np.mean(np.abs(got - ref) <= tol_pose(ref, ligs.n_atoms[lig])) >= 0.999


# ------------------------------------------------------------------------------------------------
# Screen
# ------------------------------------------------------------------------------------------------

def _screen(P, dp, ligs, search, start_scores=False, **kw):
    lib = P.DeviceLibrary(ligs)
    ds = P.DeviceSearch(search, **kw)
    r = P.screen(dp, lib, ds, start_scores=start_scores)
    torch.cuda.synchronize()
    out = {"score": r.best_score.cpu().numpy().astype(np.float64), "start": r.best_start.cpu().numpy(),
           "steps": P.steps_numpy(r.best_steps), "poses": int(r.pose_count.cpu().item()),
           "status": lib.status.cpu().numpy()}
    if start_scores:
        out["finals"] = r.start_scores.cpu().numpy().reshape(ligs.n_lig, -1).astype(np.float64)
        out["start_steps"] = P.steps_numpy(r.start_steps).reshape(ligs.n_lig, search.n_starts, -1)
    return out


def test_screen_pocket48_lib100_full(P, p48):
    W, pocket, dp, G, ligs = p48
    say("screen pocket48-lib100 (100 ligands, 512 starts, S=64) with per-start scores")
    g = _screen(P, dp, ligs, W.search, start_scores=True)
    orc = oracle.dock(pocket, G, ligs, W.search, per_start=True)
    try:
        st = check_per_start(pocket, G, ligs, W.search, g["finals"], g["start_steps"], orc)
    except AssertionError:
        bad = np.argwhere(np.abs(g["finals"] - orc["finals"]) > 1e-3 * np.maximum(1, np.abs(orc["finals"])))[:4]
        for l, p in bad:
            direct = P.score_poses(dp, P.DeviceLibrary(ligs), P.DeviceSearch(W.search), [l], [p],
                                   g["start_steps"][l, p][None]).cpu().numpy()[0]
            say(f"diverging start ({l}, {p}): GPU incremental {g['finals'][l, p]!r}, GPU from-scratch {direct!r}, "
                f"oracle {orc['finals'][l, p]!r}, GPU steps {g['start_steps'][l, p, :4]}, "
                f"oracle steps {orc['start_steps'][l, p, :4]}")
        raise
    say(f"per-start: {st}")
    assert st["agree"] >= 0.99 * st["starts"]
    assert st["agree_typical"] >= 0.999 * st["agree"]
    # internal consistency: the best is the lowest per-start final, ties to the lowest start
    assert np.array_equal(g["score"], g["finals"].min(1))
    assert np.array_equal(g["start"], np.argmin(g["finals"], 1))
    e = check_exact_and_valid(pocket, G, ligs, W.search, np.arange(ligs.n_lig), g["score"], g["start"], g["steps"])
    n_flag = check_optimal(pocket, G, ligs, W.search, np.arange(ligs.n_lig), g["score"], g["start"], orc,
                           g["finals"], g["start_steps"])
    say(f"best: rescoring max rel err {e:.3g}, {n_flag} ligands split from the oracle at near-ties")
    assert g["poses"] == oracle.pose_count(ligs.n_rot, orc["status"], W.search.n_starts, W.search.n_steps)


def test_screen_tiny_against_exhaustive(P):
    pocket = I.make_pocket(32, 4, pocket_id=9)
    G = oracle.build_grids(pocket)
    ligs = I.make_ligands(60, I.DIST_TINY, 4, stream="tiny")
    srch = I.make_search(8, 2, 8, 2.0, pocket.center)
    say("screen tiny ligands S=8 vs exhaustive")
    dp = P.DevicePocket(pocket)
    g = _screen(P, dp, ligs, srch, start_scores=True)
    orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
    check_exact_and_valid(pocket, G, ligs, srch, np.arange(ligs.n_lig), g["score"], g["start"], g["steps"])
    check_optimal(pocket, G, ligs, srch, np.arange(ligs.n_lig), g["score"], g["start"], orc, g["finals"],
                  g["start_steps"])
    nrot = ligs.n_rot
    for l in range(ligs.n_lig):
        ex, _, _ = oracle.exhaustive(pocket, G, ligs, srch, l)
        if nrot[l] <= 1:
            assert abs(g["score"][l] - ex) <= tol(ex)
        else:
            assert g["score"][l] >= ex - tol(ex)


def test_screen_edge_cases(P):
    ligs = _edge_library()
    pocket = I.make_pocket(64, 16, pocket_id=5)
    G = oracle.build_grids(pocket)
    for S in (100, 1):
        srch = I.make_search(4, 2, S, 4.0, pocket.center)
        say(f"screen edge-case library ({ligs.n_lig} ligands, n up to 129, B up to 17) S={S}")
        dp = P.DevicePocket(pocket)
        g = _screen(P, dp, ligs, srch, start_scores=True)
        st = oracle.status(ligs)
        assert np.array_equal(g["status"], st)
        assert np.all(np.isinf(g["score"][st != 0])) and np.all(g["start"][st != 0] == -1)
        sel = np.arange(ligs.n_lig)
        check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
        orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
        check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
        assert g["poses"] == oracle.pose_count(ligs.n_rot, st, srch.n_starts, S)


def test_32_atom_types(P):
    # the largest type table: grids of 32 types in both layouts and a screen whose ligands use them all
    pocket = I.make_pocket((30, 28, 26), 32, pocket_id=12)
    G = oracle.build_grids(pocket)
    ligs = I.make_ligands(24, I.DIST_DRUGLIKE, 32, stream="test")
    t_used = np.unique(np.concatenate([ligs.ligand(i)[1] for i in range(ligs.n_lig)]))
    srch = I.make_search(6, 2, 32, 2.0, pocket.center)
    for layout in (0, 1):
        say(f"32-type grids 30x28x26, layout {layout}, and a 24-ligand screen (types used: {len(t_used)})")
        dp = P.DevicePocket(pocket, layout=layout)
        g = dp.view().cpu().numpy()
        err = np.abs(g.astype(np.float64) - G) / np.maximum(1.0, np.abs(G))
        assert err.max() <= 1e-6
        r = _screen(P, dp, ligs, srch, start_scores=True)
        sel = np.arange(ligs.n_lig)
        check_exact_and_valid(pocket, G, ligs, srch, sel, r["score"], r["start"], r["steps"])
        orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
        check_optimal(pocket, G, ligs, srch, sel, r["score"], r["start"], orc, r["finals"], r["start_steps"])
    assert t_used.max() >= 16  # the upper half of the table is exercised


def test_screen_is_deterministic_and_tuning_invariant(P, p48):
    W, pocket, dp, G, ligs = p48
    sub = ligs.subset(np.arange(0, 100, 9))
    runs = []
    for kw in ({}, {"starts_per_item": 3, "waves_per_block": 1}, {"starts_per_item": 64, "waves_per_block": 8},
               {"starts_per_item": 512, "waves_per_block": 2}, {}):
        say(f"screen pocket48-lib100 subset, tuning {kw}")
        runs.append(_screen(P, dp, sub, W.search, start_scores=True, **kw))
    for r in runs[1:]:
        for key in ("score", "start", "steps", "finals", "start_steps"):
            assert np.array_equal(r[key], runs[0][key]), key


@pytest.mark.parametrize("layout", [0, 1])
def test_periodic_boundary_translation_covariance(P, layout):
    pocket = I.make_pocket(40, 4, pocket_id=11)
    G = oracle.build_grids(pocket)
    ligs = I.make_ligands(16, I.DIST_DRUGLIKE, 4, stream="test")
    srch = I.make_search(4, 3, 16, 3.0, pocket.center)
    say(f"periodic boundary, layout {layout}: GPU vs oracle and roll covariance")
    dp = P.DevicePocket(pocket, boundary=1, layout=layout)
    lib = P.DeviceLibrary(ligs)
    rng = np.random.default_rng(5)
    n = 400
    lig, start = rng.integers(0, 16, n), rng.integers(0, srch.n_starts, n)
    steps = rng.integers(0, 16, (n, 12))
    base = P.score_poses(dp, lib, P.DeviceSearch(srch), lig, start, steps).cpu().numpy()
    ref = oracle.score_poses(pocket, G, ligs, srch, lig, start, steps, periodic=True)
    assert np.all(np.abs(base - ref) <= tol_pose(ref, ligs.n_atoms[lig]))
    h = pocket.spacing
    for axis_d, axis_t, k in ((0, 3, 2), (1, 2, -3), (2, 1, 5)):
        shifted = I.Search(srch.quat, srch.trans + np.float32(h * k) * np.eye(3, dtype=np.float32)[axis_d],
                           srch.n_steps)
        moved = P.score_poses(dp, lib, P.DeviceSearch(shifted), lig, start, steps).cpu().numpy()
        rolled = P.DevicePocket(pocket, boundary=1, layout=layout)
        if layout == 1:  # rolling the wrapped xy4 records gives the records of the rolled grid
            rolled.write_records(torch.roll(dp.records(), -k, dims=axis_t))
        else:
            rolled.grids.copy_(torch.roll(dp.view(), -k, dims=axis_t).reshape(-1))
        at_rolled = P.score_poses(rolled, lib, P.DeviceSearch(srch), lig, start, steps).cpu().numpy()
        assert np.all(np.abs(moved - at_rolled) <= tol_pose(at_rolled, ligs.n_atoms[lig]))
    full = I.Search(srch.quat, srch.trans + np.float32(h * 40) * np.ones(3, np.float32), srch.n_steps)
    wrapped = P.score_poses(dp, lib, P.DeviceSearch(full), lig, start, steps).cpu().numpy()
    assert np.all(np.abs(wrapped - base) <= tol_pose(base, ligs.n_atoms[lig]))


@pytest.mark.parametrize("boundary", [0, 1])
def test_layouts_give_identical_screens(P, p48, boundary):
    W, pocket, _, _, ligs = p48
    sub = ligs.subset(np.arange(0, 100, 7))
    runs, poses = [], []
    rng = np.random.default_rng(2)
    lig, start = rng.integers(0, sub.n_lig, 300), rng.integers(0, W.search.n_starts, 300)
    steps = rng.integers(0, W.search.n_steps, (300, 12))
    for layout in (0, 1):
        say(f"screen pocket48-lib100 subset, boundary {boundary}, layout {layout}")
        dp = P.DevicePocket(pocket, boundary=boundary, layout=layout)
        runs.append(_screen(P, dp, sub, W.search, start_scores=True))
        poses.append(P.score_poses(dp, P.DeviceLibrary(sub), P.DeviceSearch(W.search), lig, start, steps).cpu())
    for key in ("score", "start", "steps", "finals", "start_steps"):
        assert np.array_equal(runs[0][key], runs[1][key]), key
    assert torch.equal(poses[0], poses[1])


# ------------------------------------------------------------------------------------------------
# Top-k
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,with_ids", [(1, 1, False), (5, 5, True), (1000, 10, False), (1025, 1000, True),
                                          (70001, 1000, False), (300000, 9000, True)])
def test_topk_vs_oracle(P, n, k, with_ids):
    rng = np.random.default_rng(n)
    s = rng.integers(-50, 50, n).astype(np.float32) / 4  # many exact ties
    s[rng.integers(0, n, max(1, n // 50))] = np.inf
    s[rng.integers(0, n, max(1, n // 70))] = np.nan
    if n > 1:
        s[0] = -0.0
    ids = rng.permutation(n).astype(np.int32) + 7 if with_ids else None
    say(f"topk n={n} k={k} ids={with_ids}")
    dev_s = torch.from_numpy(s).cuda()
    dev_i = torch.from_numpy(ids).cuda() if with_ids else None
    got_s, got_i = P.topk(dev_s, k, dev_i)
    ref_s, ref_i = oracle.topk(np.where(s == 0, 0.0, s), k, ids)
    assert np.array_equal(got_i.cpu().numpy(), ref_i)
    assert np.array_equal(got_s.cpu().numpy(), np.where(np.isnan(ref_s), np.inf, ref_s).astype(np.float32))


@pytest.mark.parametrize("n_pockets,n", [(1, 5), (4, 70001)])
def test_merge_pockets_vs_definition(P, n_pockets, n):
    rng = np.random.default_rng(n)
    s = rng.integers(-20, 20, (n_pockets, n)).astype(np.float32) / 2  # many exact ties across pockets
    s[rng.random((n_pockets, n)) < 0.05] = np.inf
    s[rng.random((n_pockets, n)) < 0.02] = np.nan
    s[:, :3] = np.inf  # ligands docked nowhere
    say(f"merge {n_pockets} pockets x {n} ligands")
    best, pocket = P.merge_pockets(torch.from_numpy(s).cuda())
    t = np.where(np.isnan(s), np.inf, s)
    ref_p = np.argmin(t, axis=0)  # the first row among equal minima
    ref_b = t[ref_p, np.arange(n)]
    ref_p = np.where(np.isinf(ref_b), -1, ref_p)
    assert np.array_equal(best.cpu().numpy(), ref_b) and np.array_equal(pocket.cpu().numpy(), ref_p)


# ------------------------------------------------------------------------------------------------
# Full-size configuration 2 (96^3 x 16 grid, 256 x 32 starts, S = 256) on a stratified sample
# ------------------------------------------------------------------------------------------------

@pytest.mark.timeout(600)
def test_pocket96_lib100k_sample_full_search(P):
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    lib_all = W.ligands(n_lig=20000)
    n, b = lib_all.n_atoms, lib_all.n_rot
    rng = np.random.default_rng(11)
    # optimality sample, stratified: the largest and smallest ligands, the most and the fewest
    # torsions, small flexible ligands and typical (median-sized) ones
    med = np.flatnonzero((np.abs(n - np.median(n)) <= 2) & (np.abs(b - np.median(b)) <= 1))
    strata = [np.flatnonzero(n == n.max())[:1], np.flatnonzero(n == n.min())[:1],
              np.flatnonzero(b == 12)[:3], np.flatnonzero(b == 0)[:2],
              np.flatnonzero((b >= 2) & (n <= 17))[:2], rng.choice(med, 8, replace=False)]
    opt = np.unique(np.concatenate(strata))
    assert len(opt) >= 16
    pick = set(rng.choice(20000, 40, replace=False).tolist()) | set(opt.tolist())
    sel = np.array(sorted(pick))
    ligs = lib_all.subset(sel)
    say(f"pocket96-lib100k sample of {len(sel)} ligands ({len(opt)} for optimality: n {n[opt].min()}-{n[opt].max()}, "
        f"B {b[opt].min()}-{b[opt].max()}), 96^3 grid, full search, bench launch configuration")
    dp = P.DevicePocket(pocket)
    g = _screen(P, dp, ligs, W.search, start_scores=True, starts_per_item=256, waves_per_block=4)
    G = oracle.build_grids(pocket)  # the oracle's own grid
    e = check_exact_and_valid(pocket, G, ligs, W.search, np.arange(len(sel)), g["score"], g["start"], g["steps"])
    say(f"pocket96 sample: rescoring max rel err {e:.3g}")
    loc = np.searchsorted(sel, opt)
    orc = oracle.dock(pocket, G, ligs, W.search, sel=loc, per_start=True)
    n_div = check_optimal(pocket, G, ligs, W.search, loc, g["score"][loc], g["start"][loc], orc, g["finals"][loc],
                          g["start_steps"][loc], max_diverged=0.1)
    say(f"pocket96 optimality: {len(loc)} ligands, {n_div} split from the oracle at near-ties")
    assert g["poses"] == oracle.pose_count(ligs.n_rot, g["status"], W.search.n_starts, W.search.n_steps)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("pi,pick", [(3, "heavy"), (1, "mixed"), (0, "mixed"), (2, "heavy")])
def test_pockets4_pockets_against_the_oracle(P, pi, pick):
    """Every pocket of the 250k-ligand workload against the oracle on its own grids, full 8192-start
    search: the 128^3 and 96^3 pockets (x 16 types) with two heavy-tail ligands (80-120 atoms) each,
    the 80^3 and 64^3 pockets with one heavy-tail and two typical ligands each."""
    W = I.workload("pockets4-lib250k")
    pocket = W.pockets[pi]
    assert pocket.dims == ((64, 64, 64), (80, 80, 80), (96, 96, 96), (128, 128, 128))[pi]
    lib_all = W.ligands(n_lig=2000)
    heavy = np.flatnonzero((lib_all.n_atoms >= 80) & (lib_all.n_rot >= 4))
    typical = np.flatnonzero((np.abs(lib_all.n_atoms - 35) <= 3) & (lib_all.n_rot == 5))
    # ligands of their own per pocket: heavy-tail ones 0-1 and 3-4 alone, 2 and 5 beside two typical ones
    h0, t0 = {3: (0, 0), 1: (2, 0), 2: (3, 0), 0: (5, 2)}[pi]
    sel = heavy[h0:h0 + 2] if pick == "heavy" else np.sort(np.r_[heavy[h0:h0 + 1], typical[t0:t0 + 2]])
    assert len(sel) == (2 if pick == "heavy" else 3)
    ligs = lib_all.subset(sel)
    say(f"pockets4 {pocket.dims[0]}^3 pocket, ligands {sel.tolist()} (n {ligs.n_atoms.tolist()}, "
        f"B {ligs.n_rot.tolist()}), full search")
    dp = P.DevicePocket(pocket)
    g = _screen(P, dp, ligs, W.search, start_scores=True)
    G = oracle.build_grids(pocket)
    sel = np.arange(ligs.n_lig)
    e = check_exact_and_valid(pocket, G, ligs, W.search, sel, g["score"], g["start"], g["steps"])
    orc = oracle.dock(pocket, G, ligs, W.search, per_start=True)
    n_div = check_optimal(pocket, G, ligs, W.search, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    say(f"{pocket.dims[0]}^3: rescoring max rel err {e:.3g}, best {g['score'].tolist()} vs oracle "
        f"{orc['best'].tolist()}, {n_div} split at near-ties")


@pytest.mark.parametrize("S", [300, 1024])
def test_screen_many_steps(P, S):
    # 300 steps: five 64-lane angle groups per lane; 1024 (the limit): sixteen
    pocket = I.make_pocket(40, 4, pocket_id=13)
    G = oracle.build_grids(pocket)
    ligs = I.make_ligands(6, I.DIST_DRUGLIKE, 4, stream="test", first_id=3000)
    srch = I.make_search(4, 2, S, 3.0, pocket.center)
    say(f"screen 6 ligands, 8 starts, S={S}")
    dp = P.DevicePocket(pocket)
    g = _screen(P, dp, ligs, srch, start_scores=True)
    orc = oracle.dock(pocket, G, ligs, srch, per_start=True)
    st = check_per_start(pocket, G, ligs, srch, g["finals"], g["start_steps"], orc)
    say(f"per-start: {st}")
    assert st["agree"] >= 0.95 * st["starts"]
    sel = np.arange(ligs.n_lig)
    check_exact_and_valid(pocket, G, ligs, srch, sel, g["score"], g["start"], g["steps"])
    check_optimal(pocket, G, ligs, srch, sel, g["score"], g["start"], orc, g["finals"], g["start_steps"])
    assert np.all(g["steps"] < S)


def test_start_selection_at_full_size(P):
    import dataclasses
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    ligs = W.ligands(n_lig=200).subset(np.array([3, 50, 121, 199]))
    srch = dataclasses.replace(W.search, sweep_top=256)
    QT = srch.n_starts
    say("sweep_top 256 of 8192 starts, 4 ligands of the 100k workload")
    dp = P.DevicePocket(pocket)
    G = oracle.build_grids(pocket)
    g = _screen(P, dp, ligs, srch, start_scores=True)
    searched = np.isfinite(g["finals"])
    assert np.all(searched.sum(1) == 256)
    for l in range(ligs.n_lig):
        rig = oracle.score_poses(pocket, G, ligs, srch, np.full(QT, l), np.arange(QT), np.zeros((QT, 16), int))
        lim = tol_fp32(rig, ligs.n_atoms[l], G, pocket.dims).max()
        assert rig[searched[l]].max() <= rig[~searched[l]].min() + 2 * lim
    # the searched starts' finals against the oracle's greedy from those starts
    li, pi = np.nonzero(searched)
    gs = oracle.greedy_starts(pocket, G, ligs, srch, li, pi)
    f_gpu = g["finals"][li, pi]
    bound = tol_fp32(gs["final"], ligs.n_atoms[li], G, pocket.dims)
    agree = np.abs(f_gpu - gs["final"]) <= bound
    say(f"{agree.sum()} of {len(agree)} searched starts agree; the rest must be near-tie paths")
    assert agree.mean() >= 0.98
    assert np.all(gs["gap"][~agree] < 1e-3)
    assert g["poses"] == int(np.sum(QT + 256 * ligs.n_rot * (srch.n_steps - 1)))
