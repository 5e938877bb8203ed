"""Device-side driver of the docking screen: buffers and the order of the ABI calls.

Holds PyTorch device tensors (memory and streams only) and calls the C ABI in
``dock.py``; every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np
import torch

from . import dock


def _dev(a, device, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


class DevicePocket:
    """Receptor grids built on the device by ``dock_build_grids``."""

    def __init__(self, pocket, device="cuda", boundary: int = dock.BOUNDARY_CLAMP, layout: int = dock.LAYOUT_XY4,
                 stream=None):
        self.pocket = pocket
        self.layout = layout
        self.desc = dock.grid_desc(pocket, boundary, layout)
        nbytes = dock.grid_bytes(self.desc)
        self.grids = torch.empty(nbytes // 4, dtype=torch.float32, device=device)
        self.prot_xyz = _dev(pocket.prot_xyz, device, torch.float32)
        self.prot_type = _dev(pocket.prot_type, device, torch.int32)
        dock.build_grids(self.desc, self.prot_xyz, self.prot_type, pocket.type_R, pocket.type_eps, pocket.type_q,
                         pocket.cap, pocket.r_min, pocket.coulomb_k, self.grids, stream)

    def view(self):
        """Node values as [t][z][y][x] (in the xy4 layout, component 0 of each record)."""
        nx, ny, nz = self.pocket.dims
        if self.layout == dock.LAYOUT_XY4:
            return self.records()[..., 0]
        return self.grids.view(self.pocket.n_types, nz, ny, nx)

    def _bricks(self):
        nx, ny, nz = self.pocket.dims
        return (nx + 1) // 2 * 2, (ny + 1) // 2, (nz + 1) // 2

    def records(self):
        """The xy4 records as [t][z][y][x][4] (a copy; storage is in bricks of the 1 x 2 x 2
        records of a (y, z) pair of rows, [t][z/2][y/2][x][z&1][y&1][4])."""
        assert self.layout == dock.LAYOUT_XY4
        nx, ny, nz = self.pocket.dims
        xp, by, bz = self._bricks()
        T = self.pocket.n_types
        r = self.grids.view(T, bz, by, xp, 2, 2, 4).permute(0, 1, 4, 2, 5, 3, 6)
        return r.reshape(T, 2 * bz, 2 * by, xp, 4)[:, :nz, :ny, :nx].contiguous()

    def write_records(self, rec: torch.Tensor):
        """Stores [t][z][y][x][4] records in brick order (the inverse of records())."""
        assert self.layout == dock.LAYOUT_XY4
        nx, ny, nz = self.pocket.dims
        xp, by, bz = self._bricks()
        T = self.pocket.n_types
        full = torch.zeros((T, 2 * bz, 2 * by, xp, 4), dtype=torch.float32, device=self.grids.device)
        full[:, :nz, :ny, :nx] = rec
        b = full.view(T, bz, 2, by, 2, xp, 4).permute(0, 1, 3, 5, 2, 4, 6)
        self.grids.copy_(b.reshape(-1))


class DeviceLibrary:
    """A ligand library copied to the device and packed by ``dock_pack_ligands``."""

    def __init__(self, ligs, device="cuda", stream=None):
        self.n_lig = ligs.n_lig
        self.n_atoms = int(ligs.atom_off[-1])
        self.n_types = ligs.n_types
        self.atom_off = _dev(ligs.atom_off, device, torch.int32)
        self.xyz = _dev(ligs.xyz.reshape(-1), device, torch.float32)
        self.types = _dev(ligs.types, device, torch.uint8)
        self.bond_off = _dev(ligs.bond_off, device, torch.int32)
        self.bonds = _dev(ligs.bonds.reshape(-1), device, torch.int32)
        self.rot = _dev(ligs.rot, device, torch.uint8)
        if self.bonds.numel() == 0:  # keep valid pointers for libraries of single atoms
            self.bonds = torch.zeros(2, dtype=torch.int32, device=device)
            self.rot = torch.zeros(1, dtype=torch.uint8, device=device)
        nbytes = dock.pack_bytes(self.n_lig, self.n_atoms, self.n_types)
        self.pack = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.status = torch.empty(self.n_lig, dtype=torch.int32, device=device)
        dock.pack_ligands(self.atom_off, self.xyz, self.types, self.bond_off, self.bonds, self.rot, self.n_types,
                          self.pack, self.status, stream)

    def descriptors(self) -> dict:
        """Per-ligand (n, B, status, sum of moving-set sizes, clash pairs) as written by the packer.
        The packed library opens with an array of 32-byte records of eight int32."""
        raw = self.pack[:32 * self.n_lig].cpu().numpy().view(np.int32).reshape(self.n_lig, 8)
        return {"n": raw[:, 1].copy(), "B": raw[:, 2].copy(), "status": raw[:, 3].copy(),
                "sum_m": raw[:, 4].copy(), "n_pairs": raw[:, 5].copy()}


class DeviceSearch:
    def __init__(self, search, device="cuda", starts_per_item: int = 0, waves_per_block: int = 0):
        self.search = search
        self.quat = _dev(search.quat, device, torch.float32)
        self.trans = _dev(search.trans, device, torch.float32)
        R = int(getattr(search, "restarts", 0))
        self.init_steps = None
        if R:
            init = np.zeros((R, dock.MAX_TORSIONS), np.int32)
            given = np.asarray(search.init_steps, dtype=np.int32).reshape(R, -1)
            init[:, :given.shape[1]] = given
            self.init_steps = _dev(init, device, torch.int32)
        self.desc = dock.search_desc(self.quat, self.trans, search.n_steps, search.clash_cut, search.clash_w,
                                     starts_per_item, waves_per_block, search.sweep_top, search.passes,
                                     self.init_steps)

    @property
    def n_starts(self) -> int:
        """Rigid starts Q T."""
        return self.quat.shape[0] * self.trans.shape[0]

    @property
    def n_searched(self) -> int:
        """Searched starts: the rigid starts and their torsion restarts."""
        return self.n_starts * (1 + (0 if self.init_steps is None else self.init_steps.shape[0]))

    def desc_fields(self) -> dict:
        """The search's parameters, with a hash of its start sets (identifies the search in a manifest)."""
        h = hashlib.sha256()
        for t in (self.quat, self.trans) + (() if self.init_steps is None else (self.init_steps,)):
            h.update(t.cpu().numpy().tobytes())
        d = self.desc
        return {"n_quat": d.n_quat, "n_trans": d.n_trans, "n_steps": d.n_steps, "clash_cut": d.clash_cut,
                "clash_w": d.clash_w, "sweep_top": d.sweep_top, "passes": d.passes, "restarts": d.restarts,
                "starts": h.hexdigest()[:16]}


@dataclass
class ScreenResult:
    best_score: torch.Tensor   # float32 [n_lig]
    best_start: torch.Tensor   # int32 [n_lig]
    best_steps: torch.Tensor   # uint16 [n_lig, 16] (as int32 view on the host)
    pose_count: torch.Tensor   # uint64 [1] (int64 storage)
    start_scores: torch.Tensor | None
    start_steps: torch.Tensor | None = None


class Screener:
    """Runs ``dock_screen`` for one (pocket, library, search) with preallocated outputs."""

    def __init__(self, pocket: DevicePocket, lib: DeviceLibrary, search: DeviceSearch, start_scores: bool = False):
        self.pocket, self.lib, self.search = pocket, lib, search
        dev = pocket.grids.device
        n = lib.n_lig
        self.ws = torch.empty(dock.screen_ws_bytes(pocket.desc, n, lib.n_atoms, search.desc), dtype=torch.uint8,
                              device=dev)
        self.best_score = torch.empty(n, dtype=torch.float32, device=dev)
        self.best_start = torch.empty(n, dtype=torch.int32, device=dev)
        self.best_steps = torch.empty(n * dock.MAX_TORSIONS, dtype=torch.int16, device=dev)
        self.pose_count = torch.empty(1, dtype=torch.int64, device=dev)
        self.start_scores = (torch.empty(n * search.n_searched, dtype=torch.float32, device=dev)
                             if start_scores else None)
        self.start_steps = (torch.empty(n * search.n_searched * dock.MAX_TORSIONS, dtype=torch.int16, device=dev)
                            if start_scores else None)

    def run(self, stream=None) -> ScreenResult:
        dock.screen(self.pocket.desc, self.pocket.grids, self.lib.pack, self.lib.n_lig, self.lib.n_atoms,
                    self.search.desc, self.best_score, self.best_start, self.best_steps, self.ws,
                    self.start_scores, self.pose_count, stream, self.start_steps)
        return ScreenResult(self.best_score, self.best_start, self.best_steps.view(self.lib.n_lig, -1),
                            self.pose_count, self.start_scores, self.start_steps)


def screen(pocket: DevicePocket, lib: DeviceLibrary, search: DeviceSearch, start_scores: bool = False):
    return Screener(pocket, lib, search, start_scores).run()


def topk(scores: torch.Tensor, k: int, ids: torch.Tensor | None = None, stream=None):
    n = scores.numel()
    dev = scores.device
    ws = torch.empty(dock.topk_ws_bytes(n, k), dtype=torch.uint8, device=dev)
    out_s = torch.empty(k, dtype=torch.float32, device=dev)
    out_i = torch.empty(k, dtype=torch.int32, device=dev)
    dock.topk(scores, k, out_s, out_i, ws, ids, stream)
    return out_s, out_i


@dataclass
class RescoreResult:
    pose_start: torch.Tensor    # [n_lig, n_keep] int32 (-1: no pose)
    pose_steps: torch.Tensor    # [n_lig, n_keep, 16] int16 (total turns)
    pose_score: torch.Tensor    # [n_lig, n_keep] docking score
    pose_rescore: torch.Tensor  # [n_lig, n_keep] (NaN: dropped or absent)
    best_rescore: torch.Tensor  # [n_lig]
    best_pose: torch.Tensor     # [n_lig] slot of the best kept pose (-1: none)
    pose_xyz: torch.Tensor | None  # [n_lig, n_keep, 128, 3] float64 when asked for


def rescore(pocket: DevicePocket, lib: DeviceLibrary, search: DeviceSearch, start_scores: torch.Tensor,
            n_keep: int = 8, rmsd_min: float = 1.0, want_xyz: bool = False, stream=None) -> RescoreResult:
    """Pose filtering and rescoring of the screen's per-start results (dock_rescore)."""
    dev = pocket.grids.device
    n = lib.n_lig
    out = RescoreResult(torch.empty((n, n_keep), dtype=torch.int32, device=dev),
                        torch.empty((n, n_keep, dock.MAX_TORSIONS), dtype=torch.int16, device=dev),
                        torch.empty((n, n_keep), dtype=torch.float32, device=dev),
                        torch.empty((n, n_keep), dtype=torch.float32, device=dev),
                        torch.empty(n, dtype=torch.float32, device=dev),
                        torch.empty(n, dtype=torch.int32, device=dev),
                        torch.zeros((n, n_keep, 128, 3), dtype=torch.float64, device=dev) if want_xyz else None)
    pk = pocket.pocket
    dock.rescore(pocket.desc, pocket.grids, lib.pack, n, lib.n_atoms, search.desc, start_scores, pocket.prot_xyz,
                 pocket.prot_type, pk.type_R, pk.type_eps, pk.type_q, pk.cap, pk.r_min, pk.coulomb_k, n_keep, rmsd_min,
                 out.pose_start, out.pose_steps, out.pose_score, out.pose_rescore, out.best_rescore, out.best_pose,
                 out.pose_xyz, stream)
    return out


def merge_pockets(scores: torch.Tensor, stream=None):
    """Each ligand's best over pockets: scores [n_pockets, n] -> (best [n], pocket index [n])."""
    scores = scores.contiguous()
    best = torch.empty(scores.shape[1], dtype=torch.float32, device=scores.device)
    pocket = torch.empty(scores.shape[1], dtype=torch.int32, device=scores.device)
    dock.merge_pockets(scores, best, pocket, stream)
    return best, pocket


def score_poses(pocket: DevicePocket, lib: DeviceLibrary, search: DeviceSearch, lig, start, steps, stream=None):
    dev = pocket.grids.device
    lig = _dev(lig, dev, torch.int32)
    start = _dev(start, dev, torch.int32)
    st = np.zeros((len(lig), dock.MAX_TORSIONS), np.int16)
    steps = np.asarray(steps).reshape(len(lig), -1)
    st[:, :steps.shape[1]] = steps
    st = _dev(st.reshape(-1), dev, torch.int16)
    out = torch.empty(len(lig), dtype=torch.float32, device=dev)
    dock.score_poses(pocket.desc, pocket.grids, lib.pack, lib.n_lig, lib.n_atoms, search.desc, lig, start, st, out,
                     stream)
    return out


def steps_numpy(best_steps: torch.Tensor) -> np.ndarray:
    """uint16 steps stored in int16 tensors -> int32 array."""
    return best_steps.cpu().numpy().astype(np.int32) & 0xFFFF
