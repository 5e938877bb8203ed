"""FP64 CPU oracle of the docking screen (ctypes wrapper over ``dock_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg call this module; the product path never imports it.  It shares no
code with the HIP path: it takes the same seeded input arrays and nothing else.

Pure-NumPy parts (the ranking step) are defined here directly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAX_ATOMS = 128
MAX_TORS = 16
MAX_PAIRS = MAX_ATOMS * (MAX_ATOMS - 1) // 2

STATUS = {0: "ok", 1: "n_atoms", 2: "type", 3: "n_bonds", 4: "bond_index", 5: "degree", 6: "not_tree",
          7: "terminal_rotatable", 8: "n_torsions"}


def build(verbose: bool = False) -> str:
    """Compiles the oracle (plain C, -O2, no fast-math, OpenMP over independent work)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH,
           os.path.join(HERE, "dock_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return LIB_PATH


class Frame(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_types", ctypes.c_int32), ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double),
                ("periodic", ctypes.c_int32), ("w_out", ctypes.c_double)]


class Potential(ctypes.Structure):
    _fields_ = [("R", ctypes.POINTER(ctypes.c_double)), ("eps", ctypes.POINTER(ctypes.c_double)),
                ("q", ctypes.POINTER(ctypes.c_double)), ("cap", ctypes.c_double), ("r_min", ctypes.c_double),
                ("coulomb_k", ctypes.c_double)]


class Library(ctypes.Structure):
    _fields_ = [("atom_off", ctypes.POINTER(ctypes.c_int32)), ("xyz", ctypes.POINTER(ctypes.c_float)),
                ("type", ctypes.POINTER(ctypes.c_uint8)), ("bond_off", ctypes.POINTER(ctypes.c_int32)),
                ("bonds", ctypes.POINTER(ctypes.c_int32)), ("rot", ctypes.POINTER(ctypes.c_uint8)),
                ("n_types", ctypes.c_int32)]


class SearchC(ctypes.Structure):
    _fields_ = [("n_quat", ctypes.c_int32), ("quat", ctypes.POINTER(ctypes.c_float)),
                ("n_trans", ctypes.c_int32), ("trans", ctypes.POINTER(ctypes.c_float)),
                ("n_steps", ctypes.c_int32), ("clash_cut", ctypes.c_double), ("clash_w", ctypes.c_double),
                ("sweep_top", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("init_steps", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        _lib = ctypes.CDLL(LIB_PATH)
        _lib.or_pair_energy.restype = ctypes.c_double
        _lib.or_pair_energy.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Potential)]
        _lib.or_rescore_pair.restype = ctypes.c_double
        _lib.or_rescore_pair.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Potential)]
    return _lib


def _p(a, ct):
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data_as(ctypes.POINTER(ct))


_F64, _F32, _I32, _I64, _U8 = ctypes.c_double, ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint8


class _Keep:
    """Keeps the NumPy arrays behind a ctypes struct alive."""

    def __init__(self, struct, *arrays):
        self.struct = struct
        self.arrays = arrays

    @property
    def ref(self):
        return ctypes.byref(self.struct)


def frame(pocket, periodic: bool = False) -> _Keep:
    nx, ny, nz = pocket.dims
    f = Frame(nx, ny, nz, pocket.n_types, (ctypes.c_double * 3)(*[float(v) for v in pocket.origin]),
              float(pocket.spacing), int(periodic), float(pocket.w_out))
    return _Keep(f)


def potential(pocket) -> _Keep:
    R = np.ascontiguousarray(pocket.type_R, dtype=np.float64)
    e = np.ascontiguousarray(pocket.type_eps, dtype=np.float64)
    q = np.ascontiguousarray(pocket.type_q, dtype=np.float64)
    p = Potential(_p(R, _F64), _p(e, _F64), _p(q, _F64), float(pocket.cap), float(pocket.r_min),
                  float(pocket.coulomb_k))
    return _Keep(p, R, e, q)


def library(ligs) -> _Keep:
    arrs = [np.ascontiguousarray(ligs.atom_off, dtype=np.int32), np.ascontiguousarray(ligs.xyz, dtype=np.float32),
            np.ascontiguousarray(ligs.types, dtype=np.uint8), np.ascontiguousarray(ligs.bond_off, dtype=np.int32),
            np.ascontiguousarray(ligs.bonds, dtype=np.int32), np.ascontiguousarray(ligs.rot, dtype=np.uint8)]
    lib = Library(_p(arrs[0], _I32), _p(arrs[1], _F32), _p(arrs[2], _U8), _p(arrs[3], _I32), _p(arrs[4], _I32),
                  _p(arrs[5], _U8), int(ligs.n_types))
    return _Keep(lib, *arrs)


def search(s) -> _Keep:
    q = np.ascontiguousarray(s.quat, dtype=np.float32)
    t = np.ascontiguousarray(s.trans, dtype=np.float32)
    R = int(getattr(s, "restarts", 0))
    init = np.zeros((max(R, 1), MAX_TORS), np.int32)
    if R:
        if int(getattr(s, "sweep_top", 0)):
            raise ValueError("torsion restarts are not combined with sweep_top")
        given = np.asarray(s.init_steps, dtype=np.int32).reshape(R, -1)
        if given.min() < 0 or given.max() >= s.n_steps:
            raise ValueError("initial turns must lie in [0, n_steps)")
        init[:, :given.shape[1]] = given
    c = SearchC(len(q), _p(q, _F32), len(t), _p(t, _F32), int(s.n_steps), float(s.clash_cut), float(s.clash_w),
                int(getattr(s, "sweep_top", 0)), int(getattr(s, "passes", 1)), R, _p(init, _I32))
    return _Keep(c, q, t, init)


# ------------------------------------------------------------------------------------------------
# Grids
# ------------------------------------------------------------------------------------------------

def pair_energy(pocket, r: float, a: int, b: int) -> float:
    pot = potential(pocket)
    return _load().or_pair_energy(float(r), int(a), int(b), ctypes.pointer(pot.struct))


def build_grids(pocket, want64: bool = False):
    """Receptor grids [T, nz, ny, nx]: FP32 as stored (and the FP64 values if asked)."""
    nx, ny, nz = pocket.dims
    g32 = np.zeros((pocket.n_types, nz, ny, nx), dtype=np.float32)
    g64 = np.zeros((pocket.n_types, nz, ny, nx), dtype=np.float64) if want64 else None
    f, pot = frame(pocket), potential(pocket)
    xyz = np.ascontiguousarray(pocket.prot_xyz, dtype=np.float32)
    typ = np.ascontiguousarray(pocket.prot_type, dtype=np.int32)
    _load().or_build_grids(f.ref, pot.ref, _p(xyz, _F32), _p(typ, _I32), len(typ), _p(g32, _F32),
                           _p(g64, _F64) if want64 else None)
    return (g32, g64) if want64 else g32


def grid_nodes(pocket, tijk: np.ndarray) -> np.ndarray:
    """FP64 grid values at nodes given as rows (t, i, j, k)."""
    tijk = np.ascontiguousarray(tijk, dtype=np.int32).reshape(-1, 4)
    out = np.zeros(len(tijk), dtype=np.float64)
    f, pot = frame(pocket), potential(pocket)
    xyz = np.ascontiguousarray(pocket.prot_xyz, dtype=np.float32)
    typ = np.ascontiguousarray(pocket.prot_type, dtype=np.int32)
    _load().or_grid_nodes(f.ref, pot.ref, _p(xyz, _F32), _p(typ, _I32), len(typ), ctypes.c_int64(len(tijk)),
                          _p(tijk, _I32), _p(out, _F64))
    return out


def lookup_points(pocket, G: np.ndarray, types, X, periodic: bool = False) -> np.ndarray:
    """Interpolated value (plus restraint in clamp mode) of grid types[i] at X[i]."""
    t = np.ascontiguousarray(types, dtype=np.int32).reshape(-1)
    x = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
    G = np.ascontiguousarray(G, dtype=np.float32)
    out = np.zeros(len(t), dtype=np.float64)
    _load().or_lookup_points(frame(pocket, periodic).ref, _p(G, _F32), ctypes.c_int64(len(t)), _p(t, _I32),
                             _p(x, _F64), _p(out, _F64))
    return out


# ------------------------------------------------------------------------------------------------
# Topology, motions, score
# ------------------------------------------------------------------------------------------------

def topology(ligs, l: int) -> dict:
    lib = library(ligs)
    st, B, npairs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ta = np.zeros(MAX_TORS, np.int32)
    tb = np.zeros(MAX_TORS, np.int32)
    tbond = np.zeros(MAX_TORS, np.int32)
    mv = np.zeros((MAX_TORS, MAX_ATOMS), np.uint8)
    core = np.zeros(MAX_ATOMS, np.uint8)
    pairs = np.zeros((MAX_PAIRS, 2), np.int32)
    xref = np.zeros((MAX_ATOMS, 3), np.float64)
    _load().or_topology(lib.ref, ctypes.c_int64(l), ctypes.byref(st), ctypes.byref(B), _p(ta, _I32), _p(tb, _I32),
                        _p(tbond, _I32), _p(mv, _U8), _p(core, _U8), ctypes.byref(npairs), _p(pairs, _I32),
                        _p(xref, _F64))
    n = int(ligs.atom_off[l + 1] - ligs.atom_off[l])
    B = B.value
    return {"status": st.value, "B": B, "tor_a": ta[:B].copy(), "tor_b": tb[:B].copy(),
            "tor_bond": tbond[:B].copy(), "moving": mv[:B, :n].astype(bool), "core": core[:n].astype(bool),
            "pairs": pairs[:npairs.value].copy(), "xref": xref[:n].copy()}


def status(ligs) -> np.ndarray:
    lib = library(ligs)
    out = np.zeros(ligs.n_lig, np.int32)
    _load().or_status(lib.ref, ctypes.c_int64(ligs.n_lig), _p(out, _I32))
    return out


def quat_matrix(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    R = np.zeros(9, np.float64)
    _load().or_quat_matrix_c(_p(q, _F64), _p(R, _F64))
    return R.reshape(3, 3)


def rodrigues(u, th: float, v) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(3, np.float64)
    _load().or_rodrigues_c(_p(u, _F64), ctypes.c_double(th), _p(v, _F64), _p(out, _F64))
    return out


def _check(ligs, srch, lig, start):
    """Ligand and start indices must lie in the library and the start set (the C code trusts them)."""
    lig, start = np.atleast_1d(lig), np.atleast_1d(start)
    if lig.size and (lig.min() < 0 or lig.max() >= ligs.n_lig):
        raise ValueError("ligand index outside the library")
    qt = len(srch.quat) * len(srch.trans) * (1 + int(getattr(srch, "restarts", 0)))
    if start.size and (start.min() < 0 or start.max() >= qt):
        raise ValueError(f"start index outside the {qt} searched starts")


def pose_coords(ligs, srch, l: int, p: int, steps=(), upto: int = MAX_TORS) -> np.ndarray:
    _check(ligs, srch, l, p)
    lib, s = library(ligs), search(srch)
    st = np.zeros(MAX_TORS, np.int32)
    st[:len(steps)] = steps
    n = int(ligs.atom_off[l + 1] - ligs.atom_off[l])
    X = np.zeros((MAX_ATOMS, 3), np.float64)
    _load().or_pose_coords(lib.ref, s.ref, ctypes.c_int64(l), ctypes.c_int32(p), _p(st, _I32), ctypes.c_int32(upto),
                           _p(X, _F64))
    return X[:n].copy()


def score_conformer(pocket, G, ligs, srch, l: int, X, periodic: bool = False) -> float:
    lib, s = library(ligs), search(srch)
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float32)
    out = ctypes.c_double()
    _load().or_score_conformer(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int64(l),
                               _p(X, _F64), ctypes.byref(out))
    return out.value


# ------------------------------------------------------------------------------------------------
# Search
# ------------------------------------------------------------------------------------------------

def dock(pocket, G, ligs, srch, sel=None, per_start: bool = False, periodic: bool = False) -> dict:
    """Greedy multi-start docking of the selected ligands (all by default)."""
    sel = np.arange(ligs.n_lig, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    lib, s = library(ligs), search(srch)
    G = np.ascontiguousarray(G, dtype=np.float32)
    n = len(sel)
    QT = srch.n_searched
    best = np.zeros(n, np.float64)
    bp = np.zeros(n, np.int32)
    bs = np.zeros((n, MAX_TORS), np.int32)
    st = np.zeros(n, np.int32)
    fin = np.zeros((n, QT), np.float64) if per_start else None
    ss = np.zeros((n, QT, MAX_TORS), np.int32) if per_start else None
    gap = np.zeros((n, QT), np.float64) if per_start else None
    _load().or_dock(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int32(n), _p(sel, _I64),
                    _p(best, _F64), _p(bp, _I32), _p(bs, _I32), _p(st, _I32),
                    _p(fin, _F64) if per_start else None, _p(ss, _I32) if per_start else None,
                    _p(gap, _F64) if per_start else None)
    out = {"best": best, "start": bp, "steps": bs, "status": st, "sel": sel}
    if per_start:
        out.update(finals=fin, start_steps=ss, start_gap=gap)
    return out


def greedy_starts(pocket, G, ligs, srch, lig, start, periodic: bool = False) -> dict:
    lig = np.ascontiguousarray(lig, dtype=np.int64)
    start = np.ascontiguousarray(start, dtype=np.int32)
    _check(ligs, srch, lig, start)
    n = len(lig)
    lib, s = library(ligs), search(srch)
    G = np.ascontiguousarray(G, dtype=np.float32)
    fin = np.zeros(n, np.float64)
    steps = np.zeros((n, MAX_TORS), np.int32)
    gap = np.zeros(n, np.float64)
    _load().or_greedy_starts(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int64(n),
                             _p(lig, _I64), _p(start, _I32), _p(fin, _F64), _p(steps, _I32), _p(gap, _F64))
    return {"final": fin, "steps": steps, "gap": gap}


def score_poses(pocket, G, ligs, srch, lig, start, steps, periodic: bool = False) -> np.ndarray:
    lig = np.ascontiguousarray(lig, dtype=np.int64)
    start = np.ascontiguousarray(start, dtype=np.int32)
    _check(ligs, srch, lig, start)
    st = np.zeros((len(lig), MAX_TORS), np.int32)
    steps = np.asarray(steps, dtype=np.int32).reshape(len(lig), -1)
    st[:, :steps.shape[1]] = steps
    lib, s = library(ligs), search(srch)
    G = np.ascontiguousarray(G, dtype=np.float32)
    out = np.zeros(len(lig), np.float64)
    _load().or_score_poses(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int64(len(lig)),
                           _p(lig, _I64), _p(start, _I32), _p(st, _I32), _p(out, _F64))
    return out


def replay(pocket, G, ligs, srch, lig, start, steps, periodic: bool = False) -> dict:
    lig = np.ascontiguousarray(lig, dtype=np.int64)
    start = np.ascontiguousarray(start, dtype=np.int32)
    _check(ligs, srch, lig, start)
    st = np.zeros((len(lig), MAX_TORS), np.int32)
    steps = np.asarray(steps, dtype=np.int32).reshape(len(lig), -1)
    st[:, :steps.shape[1]] = steps
    lib, s = library(ligs), search(srch)
    G = np.ascontiguousarray(G, dtype=np.float32)
    eg = np.zeros((len(lig), MAX_TORS), np.float64)
    em = np.zeros((len(lig), MAX_TORS), np.float64)
    fin = np.zeros(len(lig), np.float64)
    _load().or_replay(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int64(len(lig)),
                      _p(lig, _I64), _p(start, _I32), _p(st, _I32), _p(eg, _F64), _p(em, _F64), _p(fin, _F64))
    return {"e_given": eg, "e_min": em, "final": fin}


def exhaustive(pocket, G, ligs, srch, l: int, periodic: bool = False):
    lib, s = library(ligs), search(srch)
    G = np.ascontiguousarray(G, dtype=np.float32)
    best = ctypes.c_double()
    bp = ctypes.c_int32()
    bs = np.zeros(MAX_TORS, np.int32)
    _load().or_exhaustive(frame(pocket, periodic).ref, _p(G, _F32), lib.ref, s.ref, ctypes.c_int64(l),
                          ctypes.byref(best), ctypes.byref(bp), _p(bs, _I32))
    return best.value, bp.value, bs


# ------------------------------------------------------------------------------------------------
# Ranking and counting
# ------------------------------------------------------------------------------------------------

def _prot(pocket):
    xyz = np.ascontiguousarray(pocket.prot_xyz, dtype=np.float32)
    t = np.ascontiguousarray(pocket.prot_type, dtype=np.int32)
    return xyz, t


def filter_rescore(pocket, ligs, srch, l: int, start, steps, rmsd_min: float) -> dict:
    """Pose filtering and rescoring of ligand l's poses (start[i], steps[i]) given in docking order."""
    lib, s, pot = library(ligs), search(srch), potential(pocket)
    xyz, t = _prot(pocket)
    start = np.ascontiguousarray(start, dtype=np.int32)
    _check(ligs, srch, l, start[start >= 0])  # start < 0 marks an absent pose
    n = len(start)
    st = np.zeros((n, MAX_TORS), np.int32)
    st[:, :np.shape(steps)[1]] = steps
    kept = np.zeros(n, np.int32)
    rescore = np.zeros(n, np.float64)
    nearest = np.zeros(n, np.float64)
    _load().or_filter_rescore(pot.ref, _p(xyz, _F32), _p(t, _I32), ctypes.c_int32(len(t)), lib.ref, s.ref,
                              ctypes.c_int64(l), ctypes.c_int32(n), _p(start, _I32), _p(st, _I32),
                              ctypes.c_double(rmsd_min), _p(kept, _I32), _p(rescore, _F64), _p(nearest, _F64))
    return {"kept": kept.astype(bool), "rescore": rescore, "nearest": nearest}


def rescore_conformer(pocket, ligs, srch, l: int, X) -> float:
    lib, s, pot = library(ligs), search(srch), potential(pocket)
    xyz, t = _prot(pocket)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = ctypes.c_double()
    _load().or_rescore_conformer(pot.ref, _p(xyz, _F32), _p(t, _I32), ctypes.c_int32(len(t)), lib.ref, s.ref,
                                 ctypes.c_int64(l), _p(X, _F64), ctypes.byref(out))
    return out.value


def rescore_pair(pocket, r: float, a: int, b: int) -> float:
    pot = potential(pocket)
    return _load().or_rescore_pair(float(r), int(a), int(b), ctypes.pointer(pot.struct))


def set_threads(n: int) -> None:
    """OpenMP threads of the batch entry points (dock, score_poses, ...)."""
    _load().or_set_threads(ctypes.c_int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def topk(scores, k: int, ids=None):
    """The k lowest scores, ties to the lower id (NaN ranks as +inf)."""
    scores = np.asarray(scores, dtype=np.float64)
    ids = np.arange(len(scores), dtype=np.int64) if ids is None else np.asarray(ids, dtype=np.int64)
    key = np.where(np.isnan(scores), np.inf, scores)
    order = np.lexsort((ids, key))[:k]
    return scores[order], ids[order]


def pose_count(n_rot, status, n_starts: int, n_steps: int) -> int:
    """Distinct poses scored: per docked ligand, starts x (1 + B (S - 1))."""
    n_rot = np.asarray(n_rot, dtype=np.int64)
    ok = np.asarray(status) == 0
    return int(np.sum(ok * n_starts * (1 + n_rot * (n_steps - 1))))
