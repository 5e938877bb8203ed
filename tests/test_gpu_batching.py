"""Bucketed, autotuned, hipGraph-replayed chunked screening equals one eager screen."""
import numpy as np
import pytest
import torch

import oracle
from parity import check_exact_and_valid
from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import batching as Bt
    from paper_2304_09953_amd import pipeline as P
    return P, Bt


@pytest.fixture(scope="module")
def uneven():
    W = I.workload("pockets4-lib250k")
    lib = W.ligands(n_lig=20000)
    n = lib.n_atoms
    rng = np.random.default_rng(4)
    pick = np.sort(np.concatenate([rng.choice(np.flatnonzero(n < 80), 700, replace=False),
                                   rng.choice(np.flatnonzero(n >= 80), 100, replace=False)]))
    return W, lib.subset(pick)


def test_graph_chunks_equal_eager_screen_on_all_pockets(env, uneven):
    P, Bt = env
    W, ligs = uneven
    k = 100
    for pi, pocket in enumerate(W.pockets):
        srch = I.search_for(pocket, W.search)
        say(f"pocket {pi} {pocket.dims}: eager screen of {ligs.n_lig} ligands (5% at 80-120 atoms)")
        dp = P.DevicePocket(pocket)
        r = P.screen(dp, P.DeviceLibrary(ligs), P.DeviceSearch(srch))
        torch.cuda.synchronize()
        eager = r.best_score.cpu().numpy()
        say(f"pocket {pi}: bucketed graph-replayed chunks")
        top_s, top_i, best = Bt.screen_buckets(dp, srch, ligs, k=k, chunk=96, tuned=False, use_graph=True)
        assert np.array_equal(best, eager)  # identical per-start arithmetic in any launch
        ref_s, ref_i = oracle.topk(eager, k, ligs.ids)
        assert np.array_equal(top_i, ref_i.astype(np.int32))
        assert np.array_equal(top_s, ref_s.astype(np.float32))


def test_graph_replays_match_eager_runs(env, uneven):
    P, Bt = env
    W, ligs = uneven
    pocket = W.pockets[0]
    srch = I.search_for(pocket, W.search)
    dp = P.DevicePocket(pocket)
    sub = ligs.subset(np.arange(64))
    shape = Bt.chunk_shape_for(sub, np.arange(64), 64)
    graph = Bt.ChunkPipeline(dp, srch, shape, sub.n_types, 16, use_graph=True)
    eager = Bt.ChunkPipeline(dp, srch, shape, sub.n_types, 16, use_graph=False)
    for rep in range(3):
        say(f"graph replay {rep} against an eager run")
        for pipe in (graph, eager):
            pipe.reset()
            pipe.load(sub, sub.ids.astype(np.int32))
            pipe.run()
            torch.cuda.synchronize()
        assert torch.equal(graph.scores, eager.scores) and torch.equal(graph.ids, eager.ids)
        _ = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays


@pytest.mark.parametrize("budget", ["top16-passes2", "restarts2"])
def test_graph_replays_of_budget_searches_match_eager(env, uneven, budget):
    # start selection (its own kernel and workspace) and restarts inside captured chunks
    import dataclasses
    P, Bt = env
    W, ligs = uneven
    pocket = W.pockets[0]
    v = dict(sweep_top=16, passes=2) if budget == "top16-passes2" else \
        dict(restarts=2, init_steps=I.restart_steps(2, W.search.n_steps))
    srch = I.search_for(pocket, dataclasses.replace(W.search, **v))
    dp = P.DevicePocket(pocket)
    sub = ligs.subset(np.arange(64))
    say(f"{budget}: eager screen of 64 ligands")
    r = P.screen(dp, P.DeviceLibrary(sub), P.DeviceSearch(srch))
    torch.cuda.synchronize()
    eager = r.best_score.cpu().numpy()
    shape = Bt.chunk_shape_for(sub, np.arange(64), 64)
    graph = Bt.ChunkPipeline(dp, srch, shape, sub.n_types, 64, use_graph=True)
    for rep in range(2):
        say(f"{budget}: graph replay {rep}")
        graph.reset()
        graph.load(sub, sub.ids.astype(np.int32))
        graph.run()
        torch.cuda.synchronize()
        assert np.array_equal(graph.scores.cpu().numpy()[64:128], eager)  # the chunk's per-ligand best
        ref_s, ref_i = oracle.topk(eager, 64, sub.ids)
        assert np.array_equal(graph.ids.cpu().numpy()[:64], ref_i.astype(np.int32))
        assert np.array_equal(graph.scores.cpu().numpy()[:64], ref_s.astype(np.float32))
        _ = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays


def test_large_pocket_parity_sample(env, uneven):
    P, Bt = env
    W, ligs = uneven
    pocket = W.pockets[0]  # 64^3: the oracle's grid is cheap enough to build here
    srch = I.search_for(pocket, W.search)
    sel = np.r_[np.flatnonzero(ligs.n_atoms >= 80)[:3], np.arange(3)]
    sub = ligs.subset(sel)
    say("64^3 pocket: oracle rescoring of 6 ligands incl. 3 with 80-120 atoms")
    dp = P.DevicePocket(pocket)
    r = P.screen(dp, P.DeviceLibrary(sub), P.DeviceSearch(srch))
    torch.cuda.synchronize()
    G = oracle.build_grids(pocket)
    check_exact_and_valid(pocket, G, sub, srch, np.arange(sub.n_lig), r.best_score.cpu().numpy().astype(np.float64),
                          r.best_start.cpu().numpy(), P.steps_numpy(r.best_steps))
    # 128^3 grid: sampled nodes
    big = W.pockets[3]
    gb = P.DevicePocket(big).view().cpu().numpy()
    rng = np.random.default_rng(1)
    tijk = np.stack([rng.integers(0, 16, 500)] + [rng.integers(0, 128, 500) for _ in range(3)], 1).astype(np.int32)
    ref = oracle.grid_nodes(big, tijk)
    assert np.all(np.abs(gb[tijk[:, 0], tijk[:, 3], tijk[:, 2], tijk[:, 1]] - ref) <= 1e-6 * np.maximum(1, np.abs(ref)))


def test_autotuner_writes_a_usable_table(env, uneven, tmp_path, monkeypatch):
    P, Bt = env
    W, ligs = uneven
    pocket = W.pockets[0]
    srch = I.search_for(pocket, W.search)
    dp = P.DevicePocket(pocket)
    small = I.Search(srch.quat[:16], srch.trans[:4], srch.n_steps)
    say("autotune a small sample")
    cands = [(32, 4), (0, 8)]  # an explicit item size, and the library's device model
    monkeypatch.setattr(Bt, "CANDIDATES", cands)
    table = Bt.autotune(dp, ligs.subset(np.arange(0, 800, 20)), small, per_bucket=8)
    path = Bt.save_table(table, "testarch", pocket.dims, small.n_steps, str(tmp_path / "t.json"))
    for b, v in table.items():
        assert (v["starts_per_item"], v["waves_per_block"]) in cands
        assert Bt.lookup("testarch", pocket.dims, small.n_steps, b, path) == (v["starts_per_item"],
                                                                               v["waves_per_block"])


def test_shared_pack_sites_equal_per_pocket_eager_screens(env, uneven):
    """One pack per chunk screened against all four pockets (each with its tuned launch parameters)
    inside one graph: every pocket's per-ligand scores and top-k, and the best-site ranking, equal
    per-pocket eager screens of the whole library bit for bit."""
    P, Bt = env
    W, ligs = uneven
    k = 100
    dps = [P.DevicePocket(p) for p in W.pockets]
    searches = [I.search_for(p, W.search) for p in W.pockets]
    eager = []
    for pi, (dp, srch) in enumerate(zip(dps, searches)):
        say(f"pocket {pi} {W.pockets[pi].dims}: eager screen of {ligs.n_lig} ligands")
        r = P.screen(dp, P.DeviceLibrary(ligs), P.DeviceSearch(srch))
        torch.cuda.synchronize()
        eager.append(r.best_score.cpu().numpy())
    eager = np.stack(eager)
    say("shared pack: four pockets per graph-replayed chunk, tuned launch parameters")
    res = Bt.screen_sites(dps, searches, ligs, k=k, chunk=96, tuned=True, use_graph=True)
    assert np.array_equal(res.best, eager)
    for pi in range(len(dps)):
        ref_s, ref_i = oracle.topk(eager[pi], k, ligs.ids)
        assert np.array_equal(res.top_i[pi], ref_i.astype(np.int32))
        assert np.array_equal(res.top_s[pi], ref_s.astype(np.float32))
    # best site: the lowest score over pockets, ties to the lower pocket; then the top k
    site = np.argmin(eager, axis=0)
    best_site = eager[site, np.arange(ligs.n_lig)]
    site = np.where(np.isinf(best_site), -1, site)
    assert np.array_equal(res.site, site.astype(np.int32))
    ref_s, ref_i = oracle.topk(best_site, k, ligs.ids)
    assert np.array_equal(res.site_top_i, ref_i.astype(np.int32))
    assert np.array_equal(res.site_top_s, ref_s.astype(np.float32))


def test_sites_graph_replays_match_eager_runs(env, uneven):
    P, Bt = env
    W, ligs = uneven
    dps = [P.DevicePocket(p) for p in W.pockets[:2]]
    searches = [I.search_for(p, W.search) for p in W.pockets[:2]]
    sub = ligs.subset(np.arange(64))
    shape = Bt.chunk_shape_for(sub, np.arange(64), 64)
    graph = Bt.SitesChunkPipeline(dps, searches, shape, sub.n_types, 16, use_graph=True)
    eager = Bt.SitesChunkPipeline(dps, searches, shape, sub.n_types, 16, use_graph=False)
    for rep in range(3):
        say(f"two-site graph replay {rep} against an eager run")
        for pipe in (graph, eager):
            pipe.reset()
            pipe.load(sub, sub.ids.astype(np.int32))
            pipe.run()
            torch.cuda.synchronize()
        for name in ("scores", "ids", "site", "site_scores", "site_ids"):
            a, b = getattr(graph, name), getattr(eager, name)
            if name == "site":
                a, b = a[16:], b[16:]  # only the chunk part of the merge is defined
            assert torch.equal(a, b), name
        _ = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays
