"""Python binding of the C ABI in ``include/ligate_dock.h`` (``libligate.so``).

Argument marshalling only: every step of the docking path runs in the HIP kernels
of the library.  Tensors are PyTorch device tensors (PyTorch supplies device memory
and streams); the library never allocates.  There is no CPU fallback: if the
library is missing or was not built, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from .build import LIB_PATH

MAX_ATOMS = 128
MAX_TORSIONS = 16
MAX_TYPES = 32
MAX_STEPS = 1024
LAYOUT_LINEAR = 0
LAYOUT_XY4 = 1
BOUNDARY_CLAMP = 0
BOUNDARY_PERIODIC = 1

LIG_STATUS = {0: "ok", 1: "n_atoms", 2: "type", 3: "n_bonds", 4: "bond_index", 5: "degree", 6: "not_tree",
              7: "terminal_rotatable", 8: "n_torsions"}

EXPORTS = ("dock_grid_bytes", "dock_build_grids", "dock_pack_ligands", "dock_screen", "dock_screen_noalloc", "dock_topk",
           "dock_merge_pockets", "dock_score_poses", "dock_rescore", "dock_error_string", "dock_last_error")


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float), ("layout", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("w_out", ctypes.c_float)]


class TypeParam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("eps", ctypes.c_double), ("q", ctypes.c_double)]


class Potential(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_double), ("r_min", ctypes.c_double), ("coulomb_k", ctypes.c_double)]


class SearchDesc(ctypes.Structure):
    _fields_ = [("n_quat", ctypes.c_int32), ("d_quat", ctypes.c_void_p), ("n_trans", ctypes.c_int32),
                ("d_trans", ctypes.c_void_p), ("n_steps", ctypes.c_int32), ("clash_cut", ctypes.c_float),
                ("clash_w", ctypes.c_float), ("starts_per_item", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("sweep_top", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("d_init_steps", ctypes.c_void_p)]


class DockError(RuntimeError):
    pass


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DockError(f"{LIB_PATH} is missing: the HIP library has not been built (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        lib.dock_grid_bytes.argtypes = [P(GridDesc), P(sz)]
        lib.dock_build_grids.argtypes = [P(GridDesc), vp, vp, i32, P(TypeParam), P(Potential), vp, vp]
        lib.dock_pack_ligands.argtypes = [vp, vp, vp, vp, vp, vp, i32, i64, i32, vp, P(sz), vp, vp]
        lib.dock_screen.argtypes = [P(GridDesc), vp, vp, i32, i64, P(SearchDesc), vp, vp, vp, vp, vp, vp, vp, P(sz), vp]
        lib.dock_screen_noalloc.argtypes = [P(GridDesc), vp, vp, i32, i64, P(SearchDesc), vp, vp, vp, vp, vp, vp,
                                            vp]
        lib.dock_topk.argtypes = [vp, vp, i64, i32, vp, vp, vp, P(sz), vp]
        lib.dock_score_poses.argtypes = [P(GridDesc), vp, vp, i32, i64, P(SearchDesc), vp, vp, vp, i64, vp, vp]
        lib.dock_merge_pockets.argtypes = [vp, i32, i64, vp, vp, vp]
        lib.dock_rescore.argtypes = [P(GridDesc), vp, vp, i32, i64, P(SearchDesc), vp, vp, vp, i32, P(TypeParam),
                                     P(Potential), i32, ctypes.c_float, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dock_error_string.restype = ctypes.c_char_p
        lib.dock_error_string.argtypes = [ctypes.c_int]
        lib.dock_last_error.restype = ctypes.c_char_p
        lib.dock_last_error.argtypes = []
        for name in EXPORTS:
            getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        lib = load()
        raise DockError(f"{what}: {lib.dock_error_string(rc).decode()} ({rc}): {lib.dock_last_error().decode()}")


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------------------------------------
# Descriptors
# ------------------------------------------------------------------------------------------------

def grid_desc(pocket, boundary: int = BOUNDARY_CLAMP, layout: int = LAYOUT_XY4) -> GridDesc:
    nx, ny, nz = pocket.dims
    return GridDesc(nx, ny, nz, pocket.n_types, (ctypes.c_float * 3)(*[float(v) for v in pocket.origin]),
                    float(pocket.spacing), layout, boundary, float(pocket.w_out))


def search_desc(d_quat: torch.Tensor, d_trans: torch.Tensor, n_steps: int, clash_cut: float = 2.5,
                clash_w: float = 10.0, starts_per_item: int = 0, waves_per_block: int = 0, sweep_top: int = 0,
                passes: int = 1, d_init_steps: torch.Tensor | None = None) -> SearchDesc:
    """d_init_steps: int32 [R][16] initial turns of R torsion restarts per rigid start (device), or None."""
    R = 0 if d_init_steps is None else d_init_steps.shape[0]
    return SearchDesc(d_quat.shape[0], d_quat.data_ptr(), d_trans.shape[0], d_trans.data_ptr(), int(n_steps),
                      float(clash_cut), float(clash_w), int(starts_per_item), int(waves_per_block), int(sweep_top),
                      int(passes), R, d_init_steps.data_ptr() if R else None)


# ------------------------------------------------------------------------------------------------
# Calls
# ------------------------------------------------------------------------------------------------

def grid_bytes(desc: GridDesc) -> int:
    out = ctypes.c_size_t()
    _check(load().dock_grid_bytes(ctypes.byref(desc), ctypes.byref(out)), "dock_grid_bytes")
    return out.value


def build_grids(desc: GridDesc, prot_xyz: torch.Tensor, prot_type: torch.Tensor, type_R, type_eps, type_q,
                cap: float, r_min: float, coulomb_k: float, out: torch.Tensor, stream=None):
    T = desc.n_types
    params = (TypeParam * T)(*[TypeParam(float(type_R[t]), float(type_eps[t]), float(type_q[t])) for t in range(T)])
    pot = Potential(float(cap), float(r_min), float(coulomb_k))
    _check(load().dock_build_grids(ctypes.byref(desc), _ptr(prot_xyz), _ptr(prot_type), prot_type.numel(), params,
                                   ctypes.byref(pot), _ptr(out), _stream(stream)), "dock_build_grids")
    return out


def rescore(desc: GridDesc, grids: torch.Tensor, pack: torch.Tensor, n_lig: int, n_atoms: int, search: SearchDesc,
            start_scores: torch.Tensor, prot_xyz: torch.Tensor, prot_type: torch.Tensor, type_R, type_eps, type_q,
            cap: float, r_min: float, coulomb_k: float, n_keep: int, rmsd_min: float, pose_start, pose_steps,
            pose_score, pose_rescore, best_rescore, best_pose, pose_xyz=None, stream=None):
    T = desc.n_types
    params = (TypeParam * T)(*[TypeParam(float(type_R[t]), float(type_eps[t]), float(type_q[t])) for t in range(T)])
    pot = Potential(float(cap), float(r_min), float(coulomb_k))
    _check(load().dock_rescore(ctypes.byref(desc), _ptr(grids), _ptr(pack), n_lig, n_atoms, ctypes.byref(search),
                               _ptr(start_scores), _ptr(prot_xyz), _ptr(prot_type), prot_type.numel(), params,
                               ctypes.byref(pot), n_keep, float(rmsd_min), _ptr(pose_start), _ptr(pose_steps),
                               _ptr(pose_score), _ptr(pose_rescore), _ptr(best_rescore), _ptr(best_pose),
                               _ptr(pose_xyz), _stream(stream)), "dock_rescore")


def pack_bytes(n_lig: int, n_atoms: int, n_types: int) -> int:
    out = ctypes.c_size_t()
    _check(load().dock_pack_ligands(None, None, None, None, None, None, n_lig, n_atoms, n_types, None,
                                    ctypes.byref(out), None, None), "dock_pack_ligands(size)")
    return out.value


def pack_ligands(atom_off, xyz, types, bond_off, bonds, rot, n_types: int, pack: torch.Tensor,
                 status: torch.Tensor, stream=None):
    n_lig = atom_off.numel() - 1
    n_atoms = types.numel()
    size = ctypes.c_size_t(pack.numel() * pack.element_size())
    _check(load().dock_pack_ligands(_ptr(atom_off), _ptr(xyz), _ptr(types), _ptr(bond_off), _ptr(bonds), _ptr(rot),
                                    n_lig, n_atoms, n_types, _ptr(pack), ctypes.byref(size), _ptr(status),
                                    _stream(stream)), "dock_pack_ligands")


def screen_ws_bytes(desc: GridDesc, n_lig: int, n_atoms: int, search: SearchDesc) -> int:
    out = ctypes.c_size_t()
    _check(load().dock_screen(ctypes.byref(desc), None, None, n_lig, n_atoms, ctypes.byref(search), None, None, None,
                              None, None, None, None, ctypes.byref(out), None), "dock_screen(size)")
    return out.value


def screen(desc: GridDesc, grids, pack, n_lig: int, n_atoms: int, search: SearchDesc, best_score, best_start,
           best_steps, ws, start_scores=None, pose_count=None, stream=None, start_steps=None):
    size = ctypes.c_size_t(ws.numel() * ws.element_size())
    _check(load().dock_screen(ctypes.byref(desc), _ptr(grids), _ptr(pack), n_lig, n_atoms, ctypes.byref(search),
                              _ptr(best_score), _ptr(best_start), _ptr(best_steps), _ptr(start_scores),
                              _ptr(start_steps), _ptr(pose_count), _ptr(ws), ctypes.byref(size), _stream(stream)),
           "dock_screen")


def screen_noalloc(desc: GridDesc, grids, pack, n_lig: int, n_atoms: int, search: SearchDesc, best_score, best_start,
                   best_steps, start_scores=None, pose_count=None, stream=None, start_steps=None):
    """dock_screen_noalloc: the screen with the library's fixed device scratch (no workspace)."""
    _check(load().dock_screen_noalloc(ctypes.byref(desc), _ptr(grids), _ptr(pack), n_lig, n_atoms,
                                      ctypes.byref(search), _ptr(best_score), _ptr(best_start), _ptr(best_steps),
                                      _ptr(start_scores), _ptr(start_steps), _ptr(pose_count), _stream(stream)),
           "dock_screen_noalloc")


def topk_ws_bytes(n: int, k: int) -> int:
    out = ctypes.c_size_t()
    _check(load().dock_topk(None, None, n, k, None, None, None, ctypes.byref(out), None), "dock_topk(size)")
    return out.value


def topk(scores, k: int, out_scores, out_ids, ws, ids=None, stream=None):
    size = ctypes.c_size_t(ws.numel() * ws.element_size())
    _check(load().dock_topk(_ptr(scores), _ptr(ids), scores.numel(), k, _ptr(out_scores), _ptr(out_ids), _ptr(ws),
                            ctypes.byref(size), _stream(stream)), "dock_topk")


def score_poses(desc: GridDesc, grids, pack, n_lig: int, n_atoms: int, search: SearchDesc, lig, start, steps,
                out, stream=None):
    _check(load().dock_score_poses(ctypes.byref(desc), _ptr(grids), _ptr(pack), n_lig, n_atoms, ctypes.byref(search),
                                   _ptr(lig), _ptr(start), _ptr(steps), lig.numel(), _ptr(out), _stream(stream)),
           "dock_score_poses")


def merge_pockets(scores: torch.Tensor, best: torch.Tensor, pocket: torch.Tensor, stream=None):
    """scores [n_pockets, n] float32 -> best [n] (lowest per column), pocket [n] (its row, ties low)."""
    _check(load().dock_merge_pockets(_ptr(scores), scores.shape[0], scores.shape[1], _ptr(best), _ptr(pocket),
                                     _stream(stream)), "dock_merge_pockets")


# ------------------------------------------------------------------------------------------------
# Peak calibration (include/ligate_calib.h): measurement helpers, not part of the method
# ------------------------------------------------------------------------------------------------

CALIB_EXPORTS = ("calib_fma_f32", "calib_cache_read")
_calib_bound = False


def _calib_lib():
    global _calib_bound
    lib = load()
    if not _calib_bound:
        lib.calib_fma_f32.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.calib_cache_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p]
        for n in CALIB_EXPORTS:
            getattr(lib, n).restype = ctypes.c_int
        _calib_bound = True
    return lib


def calib_fma_f32(blocks: int, iters: int, out: torch.Tensor, stream=None):
    """Enqueues blocks * 256 threads x iters x 16 non-packed FP32 FMA chains (32 FLOP per step)."""
    _check(_calib_lib().calib_fma_f32(blocks, iters, _ptr(out), _stream(stream)), "calib_fma_f32")


def calib_cache_read(buf: torch.Tensor, reps: int, blocks: int, out: torch.Tensor, stream=None):
    """Enqueues blocks x reps full reads of buf (16-byte loads); blocks * reps * buf bytes in all."""
    nbytes = buf.numel() * buf.element_size()
    _check(_calib_lib().calib_cache_read(_ptr(buf), nbytes, reps, blocks, _ptr(out), _stream(stream)),
           "calib_cache_read")
