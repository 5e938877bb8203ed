"""Batched screening of uneven ligand libraries (the batch redesign of the paper's §3.3).

Ligands are clustered by size into buckets; each bucket is screened in chunks of fixed capacity
whose launch parameters (rigid starts per work item, wavefronts per block) come from the
autotuner, and each chunk's pack -> screen -> top-k merge sequence is captured once into a
hipGraph and replayed with the next chunk's ligands copied into the same device buffers.  The
next chunk is prepared on the host in pinned memory while the device works on the current one
and is copied with stream-ordered asynchronous copies; results stay on the device until the
bucket ends.  Every
step runs in the library's kernels through the C ABI; this module only orders the calls, owns the
buffers and times candidate launch parameters.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import dock
from . import pipeline as P

TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")
BUCKET_EDGES = (25, 41, 71)  # atom-count buckets: <= 24, 25-40, 41-70, >= 71
# Autotuned: wavefronts per block.  Rigid starts per work item follow the library's device model
# (0: enough items for every compute unit's resident blocks to take four times over, at most 256
# per item), evaluated for the chunk actually launched.  Timings only carry over to a chunk when
# the sample is large enough to get the chunk's item size (256 starts, from about 1k ligands at
# 8192 starts on 256 compute units): on 256-ligand samples both the item size and the wavefronts
# per block picked were 1-3 % slower on 16k-ligand chunks of the four-pocket workload.
CANDIDATES = [(0, w) for w in (2, 4, 8)]
TUNE_SAMPLE = 2048  # ligands per size bucket


def size_bucket(n_atoms: np.ndarray) -> np.ndarray:
    return np.searchsorted(np.asarray(BUCKET_EDGES), np.asarray(n_atoms), side="right")


def arch_name() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001 - no device
        return "unknown"


def _key(arch: str, dims, S: int, bucket: int) -> str:
    return f"{arch}|{dims[0]}x{dims[1]}x{dims[2]}|S{S}|b{bucket}"


# ------------------------------------------------------------------------------------------------
# Autotuner
# ------------------------------------------------------------------------------------------------

def time_screen(pocket_dev, lib_dev, search, starts_per_item: int, waves_per_block: int, reps: int = 2) -> float:
    """Seconds per dock_screen launch with the given launch parameters (median of reps)."""
    ds = P.DeviceSearch(search, starts_per_item=starts_per_item, waves_per_block=waves_per_block)
    scr = P.Screener(pocket_dev, lib_dev, ds)
    scr.run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        scr.run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return float(np.median(ts))


def autotune(pocket_dev, ligs, search, per_bucket: int = TUNE_SAMPLE, log=None) -> dict:
    """Times every candidate (starts per item, waves per block) on a sample of each size bucket
    and keeps the fastest (starts per item 0 = the library's device model, applied at run time to
    the launched chunk).  Returns {bucket: {"starts_per_item", "waves_per_block", "s_per_ligand",
    "candidates": {...}}}."""
    b = size_bucket(ligs.n_atoms)
    out = {}
    rng = np.random.default_rng(0)
    for bucket in range(len(BUCKET_EDGES) + 1):
        idx = np.flatnonzero(b == bucket)
        if len(idx) == 0:
            continue
        sample = np.sort(rng.choice(idx, min(per_bucket, len(idx)), replace=False))
        lib_dev = P.DeviceLibrary(ligs.subset(sample))
        res = {}
        for p, w in CANDIDATES:
            res[f"{p}x{w}"] = time_screen(pocket_dev, lib_dev, search, p, w) / len(sample)
            if log:
                log(f"bucket {bucket}: starts/item {p}, waves/block {w}: {res[f'{p}x{w}'] * 1e6:.1f} us/ligand")
        best = min(res, key=res.get)
        p, w = (int(v) for v in best.split("x"))
        out[bucket] = {"starts_per_item": p, "waves_per_block": w, "s_per_ligand": res[best], "candidates": res,
                       "sample": int(len(sample))}
    return out


def save_table(table: dict, arch: str, dims, S: int, path: str | None = None) -> str:
    path = path or os.path.join(TUNING_DIR, f"{arch}.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for bucket, v in table.items():
        data[_key(arch, dims, S, int(bucket))] = {k: v[k] for k in ("starts_per_item", "waves_per_block",
                                                                    "s_per_ligand", "sample")}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    json.dump(data, open(path, "w"), indent=1, sort_keys=True)
    return path


def lookup(arch: str, dims, S: int, bucket: int, path: str | None = None) -> tuple[int, int]:
    """Tuned (starts_per_item, waves_per_block) or the library's defaults (0, 0)."""
    path = path or os.path.join(TUNING_DIR, f"{arch}.json")
    try:
        v = json.load(open(path))[_key(arch, dims, S, bucket)]
        return int(v["starts_per_item"]), int(v["waves_per_block"])
    except (OSError, KeyError, ValueError):
        return 0, 0


# ------------------------------------------------------------------------------------------------
# hipGraph-captured chunks
# ------------------------------------------------------------------------------------------------

@dataclass
class ChunkShape:
    n_lig: int      # ligand capacity of a chunk
    n_atoms: int    # atom capacity of a chunk


class ChunkStaging:
    """Pinned host copies of one chunk's inputs.  A chunk is written here on the host while the
    device still works on the previous chunk, then copied with stream-ordered asynchronous copies,
    so host preparation overlaps device work.  Reusing a staging area waits for its last copies."""

    def __init__(self, shape: ChunkShape):
        L, A = shape.n_lig, shape.n_atoms
        self.shape = shape
        pin = {"pin_memory": True}
        self.atom_off = torch.empty(L + 1, dtype=torch.int32, **pin)
        self.bond_off = torch.empty(L + 1, dtype=torch.int32, **pin)
        self.xyz = torch.empty(3 * A, dtype=torch.float32, **pin)
        self.types = torch.empty(A, dtype=torch.uint8, **pin)
        self.bonds = torch.empty(2 * max(A, 1), dtype=torch.int32, **pin)
        self.rot = torch.empty(max(A, 1), dtype=torch.uint8, **pin)
        self.gid = torch.empty(L, dtype=torch.int32, **pin)
        self.event = None
        self.n = self.a = self.e = 0

    def fill(self, ligs, ids: np.ndarray):
        L, A = self.shape.n_lig, self.shape.n_atoms
        n, a, e = ligs.n_lig, int(ligs.atom_off[-1]), int(ligs.bond_off[-1])
        assert n <= L and a <= A, (n, a, L, A)
        if self.event is not None:
            self.event.synchronize()  # the copies out of this area have finished
        off = self.atom_off.numpy()
        off[:n + 1] = ligs.atom_off
        off[n + 1:] = a  # unused slots: empty ligands (status n_atoms, score +inf)
        boff = self.bond_off.numpy()
        boff[:n + 1] = ligs.bond_off
        boff[n + 1:] = e
        self.xyz.numpy()[:3 * a] = ligs.xyz.reshape(-1)
        self.types.numpy()[:a] = ligs.types
        if e:
            self.bonds.numpy()[:2 * e] = ligs.bonds.reshape(-1)
            self.rot.numpy()[:e] = ligs.rot
        gid = self.gid.numpy()
        gid[:n] = ids
        gid[n:] = 2 ** 31 - 1
        self.n, self.a, self.e = n, a, e

    def upload(self, dst) -> None:
        """Asynchronous copies into a pipeline's input buffers (on the current stream, so after the
        work already queued there, which may still read the previous chunk)."""
        dst.atom_off.copy_(self.atom_off, non_blocking=True)
        dst.bond_off.copy_(self.bond_off, non_blocking=True)
        dst.xyz[:3 * self.a].copy_(self.xyz[:3 * self.a], non_blocking=True)
        dst.types[:self.a].copy_(self.types[:self.a], non_blocking=True)
        if self.e:
            dst.bonds[:2 * self.e].copy_(self.bonds[:2 * self.e], non_blocking=True)
            dst.rot[:self.e].copy_(self.rot[:self.e], non_blocking=True)
        dst.set_ids(self.gid)
        self.event = torch.cuda.Event()
        self.event.record()


class ChunkPipeline:
    """Fixed device buffers for one (pocket, launch parameters, chunk shape) and a hipGraph of
    pack -> screen -> merge of the chunk's best scores into a running top-k."""

    def __init__(self, pocket_dev, search, shape: ChunkShape, n_types: int, k: int, starts_per_item: int = 0,
                 waves_per_block: int = 0, use_graph: bool = True):
        dev = pocket_dev.grids.device
        self.pocket, self.shape, self.k, self.n_types = pocket_dev, shape, k, n_types
        L, A = shape.n_lig, shape.n_atoms
        self.atom_off = torch.zeros(L + 1, dtype=torch.int32, device=dev)
        self.bond_off = torch.zeros(L + 1, dtype=torch.int32, device=dev)
        self.xyz = torch.zeros(3 * A, dtype=torch.float32, device=dev)
        self.types = torch.zeros(A, dtype=torch.uint8, device=dev)
        self.bonds = torch.zeros(2 * max(A, 1), dtype=torch.int32, device=dev)
        self.rot = torch.zeros(max(A, 1), dtype=torch.uint8, device=dev)
        self.pack = torch.empty(dock.pack_bytes(L, A, n_types), dtype=torch.uint8, device=dev)
        self.status = torch.empty(L, dtype=torch.int32, device=dev)
        self.search = P.DeviceSearch(search, starts_per_item=starts_per_item, waves_per_block=waves_per_block)
        self.ws = torch.empty(dock.screen_ws_bytes(pocket_dev.desc, L, A, self.search.desc), dtype=torch.uint8,
                              device=dev)
        # merge buffer: [running top-k | this chunk's best scores], with global ligand ids
        self.scores = torch.full((k + L,), float("inf"), dtype=torch.float32, device=dev)
        self.ids = torch.full((k + L,), 2 ** 31 - 1, dtype=torch.int32, device=dev)
        self.best_start = torch.empty(L, dtype=torch.int32, device=dev)
        self.best_steps = torch.empty(L * dock.MAX_TORSIONS, dtype=torch.int16, device=dev)
        self.top_s = torch.empty(k, dtype=torch.float32, device=dev)
        self.top_i = torch.empty(k, dtype=torch.int32, device=dev)
        self.topk_ws = torch.empty(dock.topk_ws_bytes(k + L, k), dtype=torch.uint8, device=dev)
        self.graph = None
        if use_graph:
            self._capture()

    def _enqueue(self):
        L, A = self.shape.n_lig, self.shape.n_atoms
        dock.pack_ligands(self.atom_off, self.xyz, self.types, self.bond_off, self.bonds, self.rot, self.n_types,
                          self.pack, self.status)
        dock.screen(self.pocket.desc, self.pocket.grids, self.pack, L, A, self.search.desc, self.scores[self.k:],
                    self.best_start, self.best_steps, self.ws)
        dock.topk(self.scores, self.k, self.top_s, self.top_i, self.topk_ws, self.ids)
        self.scores[:self.k].copy_(self.top_s)
        self.ids[:self.k].copy_(self.top_i)

    def _capture(self):
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # warm-up outside the graph (first-launch host work)
            self._enqueue()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.reset()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        torch.cuda.synchronize()

    def reset(self):
        self.scores.fill_(float("inf"))
        self.ids.fill_(2 ** 31 - 1)

    def load(self, ligs, ids: np.ndarray):
        """Copies a chunk (at most the capacity) into the fixed buffers; unused ligand slots become
        empty ligands (status n_atoms, score +inf)."""
        L, A = self.shape.n_lig, self.shape.n_atoms
        n, a = ligs.n_lig, int(ligs.atom_off[-1])
        assert n <= L and a <= A, (n, a, L, A)
        off = np.full(L + 1, a, dtype=np.int32)
        off[:n + 1] = ligs.atom_off
        boff = np.full(L + 1, int(ligs.bond_off[-1]), dtype=np.int32)
        boff[:n + 1] = ligs.bond_off
        self.atom_off.copy_(torch.from_numpy(off))
        self.bond_off.copy_(torch.from_numpy(boff))
        self.xyz[:3 * a].copy_(torch.from_numpy(ligs.xyz.reshape(-1)))
        self.types[:a].copy_(torch.from_numpy(ligs.types))
        e = int(ligs.bond_off[-1])
        if e:
            self.bonds[:2 * e].copy_(torch.from_numpy(ligs.bonds.reshape(-1)))
            self.rot[:e].copy_(torch.from_numpy(ligs.rot))
        gid = np.full(L, 2 ** 31 - 1, dtype=np.int32)
        gid[:n] = ids
        self.ids[self.k:].copy_(torch.from_numpy(gid))

    def set_ids(self, gid_pinned: torch.Tensor):
        self.ids[self.k:].copy_(gid_pinned, non_blocking=True)

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self._enqueue()


def chunk_shape_for(ligs, idx: np.ndarray, chunk: int) -> ChunkShape:
    """Capacity that fits every chunk of `chunk` ligands taken in order from idx."""
    n = ligs.n_atoms[idx]
    if len(n) == 0:
        return ChunkShape(1, 1)
    sums = [int(n[s:s + chunk].sum()) for s in range(0, len(n), chunk)]
    return ChunkShape(min(chunk, len(n)), max(sums))


def screen_buckets(pocket_dev, search, ligs, k: int = 1000, chunk: int = 16384, tuned: bool = True,
                   use_graph: bool = True, log=None, table_path: str | None = None):
    """Screens a library against one pocket bucket by bucket in graph-replayed chunks, merging
    into one running top-k.  Returns (top scores, top global ids, per-ligand best scores)."""
    arch = arch_name()
    buckets = size_bucket(ligs.n_atoms)
    best = np.full(ligs.n_lig, np.inf, dtype=np.float32)
    top_s = np.full(k, np.inf, dtype=np.float32)
    top_i = np.full(k, 2 ** 31 - 1, dtype=np.int32)
    for bucket in range(len(BUCKET_EDGES) + 1):
        idx = np.flatnonzero(buckets == bucket)
        if len(idx) == 0:
            continue
        p, w = lookup(arch, pocket_dev.pocket.dims, search.n_steps, bucket, table_path) if tuned else (0, 0)
        shape = chunk_shape_for(ligs, idx, chunk)
        pipe = ChunkPipeline(pocket_dev, search, shape, ligs.n_types, k, p, w, use_graph)
        pipe.reset()
        pipe.scores[:k].copy_(torch.from_numpy(top_s))
        pipe.ids[:k].copy_(torch.from_numpy(top_i))
        staging = [ChunkStaging(shape), ChunkStaging(shape)]
        bucket_best = torch.empty(len(idx), dtype=torch.float32, device=pipe.scores.device)
        t0 = time.perf_counter()
        for c, s in enumerate(range(0, len(idx), chunk)):
            sel = idx[s:s + chunk]
            st = staging[c % 2]
            st.fill(ligs.subset(sel), ligs.ids[sel].astype(np.int32))  # overlaps the previous chunk
            st.upload(pipe)
            pipe.run()
            bucket_best[s:s + len(sel)].copy_(pipe.scores[k:k + len(sel)])
        best[idx] = bucket_best.cpu().numpy()
        torch.cuda.synchronize()
        top_s = pipe.scores[:k].cpu().numpy()
        top_i = pipe.ids[:k].cpu().numpy()
        if log:
            log(f"bucket {bucket}: {len(idx)} ligands, starts/item {p}, waves/block {w}, "
                f"{time.perf_counter() - t0:.2f} s")
    return top_s, top_i, best


# ------------------------------------------------------------------------------------------------
# Several binding sites from one pack (a ligand is ranked by its best site)
# ------------------------------------------------------------------------------------------------

class SitesChunkPipeline:
    """Fixed device buffers for one chunk shape and several pockets, and a hipGraph of: pack the chunk
    once; screen it against every pocket (each with its own tuned launch parameters); merge each
    pocket's chunk scores into that pocket's running top-k; take each ligand's best pocket with
    dock_merge_pockets and merge those into a running top-k of the best-site ranking."""

    def __init__(self, pockets_dev, searches, shape: ChunkShape, n_types: int, k: int, params=None,
                 use_graph: bool = True):
        dev = pockets_dev[0].grids.device
        n_p = len(pockets_dev)
        assert len(searches) == n_p and n_p >= 1
        params = params or [(0, 0)] * n_p
        self.pockets, self.shape, self.k, self.n_types, self.n_p = pockets_dev, shape, k, n_types, n_p
        L, A = shape.n_lig, shape.n_atoms
        self.atom_off = torch.zeros(L + 1, dtype=torch.int32, device=dev)
        self.bond_off = torch.zeros(L + 1, dtype=torch.int32, device=dev)
        self.xyz = torch.zeros(3 * A, dtype=torch.float32, device=dev)
        self.types = torch.zeros(A, dtype=torch.uint8, device=dev)
        self.bonds = torch.zeros(2 * max(A, 1), dtype=torch.int32, device=dev)
        self.rot = torch.zeros(max(A, 1), dtype=torch.uint8, device=dev)
        self.pack = torch.empty(dock.pack_bytes(L, A, n_types), dtype=torch.uint8, device=dev)
        self.status = torch.empty(L, dtype=torch.int32, device=dev)
        self.searches = [P.DeviceSearch(s, starts_per_item=p, waves_per_block=w) for s, (p, w) in zip(searches, params)]
        ws = max(dock.screen_ws_bytes(d.desc, L, A, s.desc) for d, s in zip(pockets_dev, self.searches))
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)  # the screens run in turn on one stream
        # per pocket: [running top-k | this chunk's best scores], global ligand ids beside them
        self.scores = torch.full((n_p, k + L), float("inf"), dtype=torch.float32, device=dev)
        self.ids = torch.full((n_p, k + L), 2 ** 31 - 1, dtype=torch.int32, device=dev)
        self.best_start = torch.empty((n_p, L), dtype=torch.int32, device=dev)
        self.best_steps = torch.empty((n_p, L * dock.MAX_TORSIONS), dtype=torch.int16, device=dev)
        self.top_s = torch.empty((n_p, k), dtype=torch.float32, device=dev)
        self.top_i = torch.empty((n_p, k), dtype=torch.int32, device=dev)
        self.topk_ws = torch.empty(dock.topk_ws_bytes(k + L, k), dtype=torch.uint8, device=dev)
        # best site: dock_merge_pockets over the rows [running k | chunk] (only the chunk part is used),
        # then [running top-k | chunk's best-site scores] and its top-k
        self.merged = torch.empty(k + L, dtype=torch.float32, device=dev)
        self.site = torch.empty(k + L, dtype=torch.int32, device=dev)
        self.site_scores = torch.full((k + L,), float("inf"), dtype=torch.float32, device=dev)
        self.site_ids = torch.full((k + L,), 2 ** 31 - 1, dtype=torch.int32, device=dev)
        self.site_top_s = torch.empty(k, dtype=torch.float32, device=dev)
        self.site_top_i = torch.empty(k, dtype=torch.int32, device=dev)
        self.graph = None
        if use_graph:
            self._capture()

    def _enqueue(self):
        L, A, k = self.shape.n_lig, self.shape.n_atoms, self.k
        dock.pack_ligands(self.atom_off, self.xyz, self.types, self.bond_off, self.bonds, self.rot, self.n_types,
                          self.pack, self.status)
        for p, (dp, ds) in enumerate(zip(self.pockets, self.searches)):
            dock.screen(dp.desc, dp.grids, self.pack, L, A, ds.desc, self.scores[p, k:], self.best_start[p],
                        self.best_steps[p], self.ws)
        for p in range(self.n_p):
            dock.topk(self.scores[p], k, self.top_s[p], self.top_i[p], self.topk_ws, self.ids[p])
            self.scores[p, :k].copy_(self.top_s[p])
            self.ids[p, :k].copy_(self.top_i[p])
        dock.merge_pockets(self.scores, self.merged, self.site)
        self.site_scores[k:].copy_(self.merged[k:])
        dock.topk(self.site_scores, k, self.site_top_s, self.site_top_i, self.topk_ws, self.site_ids)
        self.site_scores[:k].copy_(self.site_top_s)
        self.site_ids[:k].copy_(self.site_top_i)

    def _capture(self):
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # warm-up outside the graph (first-launch host work)
            self._enqueue()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.reset()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        torch.cuda.synchronize()

    def reset(self):
        self.scores.fill_(float("inf"))
        self.ids.fill_(2 ** 31 - 1)
        self.site_scores.fill_(float("inf"))
        self.site_ids.fill_(2 ** 31 - 1)

    def seed(self, tops, site_top):
        """Running top-k of every pocket and of the best-site ranking (host arrays) into the buffers."""
        k = self.k
        for p, (s, i) in enumerate(tops):
            self.scores[p, :k].copy_(torch.from_numpy(s))
            self.ids[p, :k].copy_(torch.from_numpy(i))
        self.site_scores[:k].copy_(torch.from_numpy(site_top[0]))
        self.site_ids[:k].copy_(torch.from_numpy(site_top[1]))

    def load(self, ligs, ids: np.ndarray):
        """Copies a chunk (at most the capacity) into the fixed buffers; unused ligand slots become
        empty ligands (status n_atoms, score +inf)."""
        L, A = self.shape.n_lig, self.shape.n_atoms
        n, a = ligs.n_lig, int(ligs.atom_off[-1])
        assert n <= L and a <= A, (n, a, L, A)
        off = np.full(L + 1, a, dtype=np.int32)
        off[:n + 1] = ligs.atom_off
        boff = np.full(L + 1, int(ligs.bond_off[-1]), dtype=np.int32)
        boff[:n + 1] = ligs.bond_off
        self.atom_off.copy_(torch.from_numpy(off))
        self.bond_off.copy_(torch.from_numpy(boff))
        self.xyz[:3 * a].copy_(torch.from_numpy(ligs.xyz.reshape(-1)))
        self.types[:a].copy_(torch.from_numpy(ligs.types))
        e = int(ligs.bond_off[-1])
        if e:
            self.bonds[:2 * e].copy_(torch.from_numpy(ligs.bonds.reshape(-1)))
            self.rot[:e].copy_(torch.from_numpy(ligs.rot))
        gid = np.full(L, 2 ** 31 - 1, dtype=np.int32)
        gid[:n] = ids
        g = torch.from_numpy(gid)
        self.ids[:, self.k:].copy_(g.unsqueeze(0).expand(self.n_p, L))
        self.site_ids[self.k:].copy_(g)

    def set_ids(self, gid_pinned: torch.Tensor):
        L = self.shape.n_lig
        self.site_ids[self.k:].copy_(gid_pinned, non_blocking=True)
        self.ids[:, self.k:].copy_(self.site_ids[self.k:].unsqueeze(0).expand(self.n_p, L))

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self._enqueue()


@dataclass
class SitesResult:
    top_s: np.ndarray       # [n_pockets, k] each pocket's top-k scores (ascending)
    top_i: np.ndarray       # [n_pockets, k] their global ligand ids
    best: np.ndarray        # [n_pockets, n_lig] every ligand's best score against every pocket
    site_top_s: np.ndarray  # [k] best-site ranking: scores
    site_top_i: np.ndarray  # [k] best-site ranking: global ids
    site: np.ndarray        # [n_lig] each ligand's best pocket (-1 if docked nowhere)


def screen_sites(pockets_dev, searches, ligs, k: int = 1000, chunk: int = 16384, tuned: bool = True,
                 use_graph: bool = True, log=None, table_path: str | None = None) -> SitesResult:
    """Screens a library against several pockets from one pack per chunk, bucket by bucket in
    graph-replayed chunks, keeping each pocket's running top-k and the running top-k of the
    best-site ranking."""
    arch = arch_name()
    n_p = len(pockets_dev)
    buckets = size_bucket(ligs.n_atoms)
    best = np.full((n_p, ligs.n_lig), np.inf, dtype=np.float32)
    site = np.full(ligs.n_lig, -1, dtype=np.int32)
    tops = [(np.full(k, np.inf, np.float32), np.full(k, 2 ** 31 - 1, np.int32)) for _ in range(n_p)]
    site_top = (np.full(k, np.inf, np.float32), np.full(k, 2 ** 31 - 1, np.int32))
    for bucket in range(len(BUCKET_EDGES) + 1):
        idx = np.flatnonzero(buckets == bucket)
        if len(idx) == 0:
            continue
        params = [lookup(arch, dp.pocket.dims, s.n_steps, bucket, table_path) if tuned else (0, 0)
                  for dp, s in zip(pockets_dev, searches)]
        shape = chunk_shape_for(ligs, idx, chunk)
        pipe = SitesChunkPipeline(pockets_dev, searches, shape, ligs.n_types, k, params, use_graph)
        pipe.reset()
        pipe.seed(tops, site_top)
        staging = [ChunkStaging(shape), ChunkStaging(shape)]
        dev = pipe.scores.device
        bucket_best = torch.empty((n_p, len(idx)), dtype=torch.float32, device=dev)
        bucket_site = torch.empty(len(idx), dtype=torch.int32, device=dev)
        t0 = time.perf_counter()
        for c, s in enumerate(range(0, len(idx), chunk)):
            sel = idx[s:s + chunk]
            st = staging[c % 2]
            st.fill(ligs.subset(sel), ligs.ids[sel].astype(np.int32))  # overlaps the previous chunk
            st.upload(pipe)
            pipe.run()
            bucket_best[:, s:s + len(sel)].copy_(pipe.scores[:, k:k + len(sel)])
            bucket_site[s:s + len(sel)].copy_(pipe.site[k:k + len(sel)])
        best[:, idx] = bucket_best.cpu().numpy()
        site[idx] = bucket_site.cpu().numpy()
        torch.cuda.synchronize()
        tops = [(pipe.scores[p, :k].cpu().numpy(), pipe.ids[p, :k].cpu().numpy()) for p in range(n_p)]
        site_top = (pipe.site_scores[:k].cpu().numpy(), pipe.site_ids[:k].cpu().numpy())
        if log:
            log(f"bucket {bucket}: {len(idx)} ligands x {n_p} pockets, launch parameters {params}, "
                f"{time.perf_counter() - t0:.2f} s")
    return SitesResult(np.stack([t[0] for t in tops]), np.stack([t[1] for t in tops]), best, site_top[0],
                       site_top[1], site)
