"""Seeded synthetic inputs for the docking screen.

This module draws inputs only; it holds none of the docking arithmetic.  Both
the HIP path and the CPU oracle consume the arrays it returns.  The heavy lifting
(tree-shaped 3D ligands) is in ``gen.c`` (built into ``libligate_inputs.so``);
every ligand has its own counter-keyed random stream, so ligand ``g`` of a
library is the same whichever chunk it is generated in.

Workloads (synthetic stand-ins for the screening campaigns of §2 and the
batched, uneven libraries of §3.3):

* ``pocket48-lib100``: one 48^3 pocket with 8 atom types, 100 ligands of
  exactly 24 atoms and 4 rotatable bonds; 64 quaternions x 8 translations,
  64 torsion steps.
* ``pocket96-lib100k``: one 96^3 pocket with 16 types, 100k ligands with atom
  counts N(35, 10) clipped to [15, 70] and Poisson(5) rotatable bonds clipped
  to [0, 12]; 256 quaternions x 32 translations, 256 steps.
* ``pockets4-lib250k``: four pockets of 64^3, 80^3, 96^3 and 128^3, 250k
  ligands of which 5 % have 80-120 atoms; the 100k-library search.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 230409953
STREAMS = {"lib": 1, "train": 2, "pocket": 3, "search": 4, "test": 5, "sample": 6, "tiny": 7}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libligate_inputs.so")
_lib = None


class _LibParams(ctypes.Structure):
    _fields_ = [
        ("n_mean", ctypes.c_double), ("n_sd", ctypes.c_double),
        ("n_min", ctypes.c_int32), ("n_max", ctypes.c_int32),
        ("tail_p", ctypes.c_double),
        ("tail_min", ctypes.c_int32), ("tail_max", ctypes.c_int32),
        ("b_mean", ctypes.c_double),
        ("b_min", ctypes.c_int32), ("b_max", ctypes.c_int32),
        ("fixed_n", ctypes.c_int32), ("fixed_b", ctypes.c_int32),
        ("n_types", ctypes.c_int32),
        ("offset_range", ctypes.c_float),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        lib.gen_ligand_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                         P(_LibParams), P(ctypes.c_int32)]
        lib.gen_ligands.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                    P(_LibParams), P(ctypes.c_int32), P(ctypes.c_float), P(ctypes.c_uint8),
                                    P(ctypes.c_int32), P(ctypes.c_uint8), P(ctypes.c_int32)]
        lib.gen_pocket_atoms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32, P(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                                         P(ctypes.c_float), P(ctypes.c_int32)]
        lib.gen_translations.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                                         P(ctypes.c_double), P(ctypes.c_float)]
        lib.gen_quaternions.argtypes = [ctypes.c_int32, P(ctypes.c_float)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ----------------------------------------------------------------------------------------------
# Library distributions
# ----------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class LibDist:
    n_mean: float = 35.0
    n_sd: float = 10.0
    n_min: int = 15
    n_max: int = 70
    tail_p: float = 0.0
    tail_min: int = 80
    tail_max: int = 120
    b_mean: float = 5.0
    b_min: int = 0
    b_max: int = 12
    fixed_n: int = 0
    fixed_b: int = -1
    offset_range: float = 10.0

    def c(self, n_types: int) -> _LibParams:
        return _LibParams(self.n_mean, self.n_sd, self.n_min, self.n_max, self.tail_p, self.tail_min,
                          self.tail_max, self.b_mean, self.b_min, self.b_max, self.fixed_n, self.fixed_b,
                          n_types, self.offset_range)


DIST_FIXED24 = LibDist(fixed_n=24, fixed_b=4)
DIST_DRUGLIKE = LibDist()
DIST_HEAVY_TAIL = LibDist(tail_p=0.05)
DIST_TINY = LibDist(n_mean=6.0, n_sd=1.5, n_min=4, n_max=8, b_mean=1.5, b_max=3)


@dataclass
class Ligands:
    """A ligand library in CSR form (the layout the packer consumes)."""
    atom_off: np.ndarray   # int32 [L+1]
    xyz: np.ndarray        # float32 [A, 3], input conformers (not centred)
    types: np.ndarray      # uint8 [A]
    bond_off: np.ndarray   # int32 [L+1]
    bonds: np.ndarray      # int32 [E, 2], local atom indices
    rot: np.ndarray        # uint8 [E], 1 = rotatable
    ids: np.ndarray        # int64 [L], global ligand ids
    n_types: int

    @property
    def n_lig(self) -> int:
        return len(self.atom_off) - 1

    @property
    def n_atoms(self) -> np.ndarray:
        return np.diff(self.atom_off)

    @property
    def n_rot(self) -> np.ndarray:
        return np.add.reduceat(self.rot.astype(np.int64), self.bond_off[:-1]) * (np.diff(self.bond_off) > 0)

    def ligand(self, i: int):
        a0, a1 = self.atom_off[i], self.atom_off[i + 1]
        b0, b1 = self.bond_off[i], self.bond_off[i + 1]
        return self.xyz[a0:a1], self.types[a0:a1], self.bonds[b0:b1], self.rot[b0:b1]

    def subset(self, idx) -> "Ligands":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.ligand(int(i)) for i in idx]
        return from_parts(parts, self.n_types, ids=self.ids[idx])


def from_parts(parts, n_types: int, ids=None) -> Ligands:
    """Builds a CSR library from a list of (xyz, types, bonds, rot) tuples."""
    n = np.array([len(p[1]) for p in parts], dtype=np.int64)
    e = np.array([len(p[3]) for p in parts], dtype=np.int64)
    atom_off = np.zeros(len(parts) + 1, dtype=np.int32)
    atom_off[1:] = np.cumsum(n)
    bond_off = np.zeros(len(parts) + 1, dtype=np.int32)
    bond_off[1:] = np.cumsum(e)
    xyz = np.zeros((int(n.sum()), 3), dtype=np.float32)
    types = np.zeros(int(n.sum()), dtype=np.uint8)
    bonds = np.zeros((int(e.sum()), 2), dtype=np.int32)
    rot = np.zeros(int(e.sum()), dtype=np.uint8)
    for i, (x, t, b, r) in enumerate(parts):
        xyz[atom_off[i]:atom_off[i + 1]] = np.asarray(x, dtype=np.float32).reshape(-1, 3)
        types[atom_off[i]:atom_off[i + 1]] = t
        if len(r):
            bonds[bond_off[i]:bond_off[i + 1]] = np.asarray(b, dtype=np.int32).reshape(-1, 2)
            rot[bond_off[i]:bond_off[i + 1]] = r
    if ids is None:
        ids = np.arange(len(parts), dtype=np.int64)
    return Ligands(atom_off, xyz, types, bond_off, bonds, rot, np.asarray(ids, dtype=np.int64), n_types)


def make_ligands(n_lig: int, dist: LibDist, n_types: int, stream: str = "lib", first_id: int = 0,
                 seed: int = BASE_SEED) -> Ligands:
    lib = _load()
    prm = dist.c(n_types)
    sid = STREAMS[stream]
    n = np.zeros(n_lig, dtype=np.int32)
    lib.gen_ligand_sizes(seed, sid, first_id, n_lig, ctypes.byref(prm), _ptr(n, ctypes.c_int32))
    atom_off = np.zeros(n_lig + 1, dtype=np.int32)
    atom_off[1:] = np.cumsum(n, dtype=np.int64)
    A = int(atom_off[-1])
    xyz = np.zeros((A, 3), dtype=np.float32)
    types = np.zeros(A, dtype=np.uint8)
    bonds = np.zeros((A - n_lig, 2), dtype=np.int32)
    rot = np.zeros(A - n_lig, dtype=np.uint8)
    nrot = np.zeros(n_lig, dtype=np.int32)
    lib.gen_ligands(seed, sid, first_id, n_lig, ctypes.byref(prm), _ptr(atom_off, ctypes.c_int32),
                    _ptr(xyz, ctypes.c_float), _ptr(types, ctypes.c_uint8), _ptr(bonds, ctypes.c_int32),
                    _ptr(rot, ctypes.c_uint8), _ptr(nrot, ctypes.c_int32))
    bond_off = (atom_off - np.arange(n_lig + 1, dtype=np.int32)).astype(np.int32)
    ids = np.arange(first_id, first_id + n_lig, dtype=np.int64)
    return Ligands(atom_off, xyz, types, bond_off, bonds, rot, ids, n_types)


# ----------------------------------------------------------------------------------------------
# Pockets
# ----------------------------------------------------------------------------------------------

@dataclass
class Pocket:
    """A rigid receptor pocket: protein atoms, the atom-type table and the grid frame."""
    dims: tuple            # (nx, ny, nz)
    n_types: int
    origin: np.ndarray     # float32 [3], a multiple of 1/8 A so node coordinates are exact
    spacing: float
    prot_xyz: np.ndarray   # float32 [N, 3]
    prot_type: np.ndarray  # int32 [N]
    type_R: np.ndarray     # float64 [T]
    type_eps: np.ndarray   # float64 [T]
    type_q: np.ndarray     # float64 [T]
    cap: float = 10.0
    r_min: float = 0.5
    coulomb_k: float = 332.0636 / 4.0
    w_out: float = 10.0

    @property
    def center(self) -> np.ndarray:
        n = np.array(self.dims, dtype=np.float64)
        return self.origin.astype(np.float64) + self.spacing * (n - 1) / 2.0

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.dims))


def type_table(n_types: int):
    """Synthetic per-type radius, well depth and charge."""
    t = np.arange(n_types, dtype=np.float64)
    return 1.50 + 0.05 * t, 0.05 + 0.01 * t, 0.2 * ((t % 4) - 1.5)


def make_pocket(dim, n_types: int, n_prot: int = 300, pocket_id: int = 0, spacing: float = 0.375,
                offset=(1.25, -0.5, 0.75), r_in: float = 6.0, r_out: float = 12.0,
                seed: int = BASE_SEED) -> Pocket:
    lib = _load()
    dims = tuple(int(d) for d in (dim if np.iterable(dim) else (dim, dim, dim)))
    half = np.array([spacing * (d - 1) / 2.0 for d in dims])
    origin = (-np.round(half * 8.0) / 8.0 + np.asarray(offset)).astype(np.float32)
    assert np.all(origin * 8 == np.round(origin * 8))
    center = origin.astype(np.float64) + half
    xyz = np.zeros((n_prot, 3), dtype=np.float32)
    typ = np.zeros(n_prot, dtype=np.int32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    lib.gen_pocket_atoms(seed, STREAMS["pocket"], pocket_id, n_prot, n_types, _ptr(c, ctypes.c_double),
                         r_in, r_out, _ptr(xyz, ctypes.c_float), _ptr(typ, ctypes.c_int32))
    R, eps, q = type_table(n_types)
    return Pocket(dims, n_types, origin, float(spacing), xyz, typ, R, eps, q)


# ----------------------------------------------------------------------------------------------
# Search sets
# ----------------------------------------------------------------------------------------------

@dataclass
class Search:
    quat: np.ndarray      # float32 [Q, 4] (w, x, y, z)
    trans: np.ndarray     # float32 [T, 3]
    n_steps: int
    clash_cut: float = 2.5
    clash_w: float = 10.0
    sweep_top: int = 0    # 0: every start gets the torsion sweeps; K: only the K best rigid starts
    passes: int = 1       # greedy passes over the torsions
    restarts: int = 0     # R torsion restarts per rigid start (not combined with sweep_top)
    init_steps: np.ndarray | None = None  # int32 [R][16]: initial turn of each torsion, in [0, n_steps)

    @property
    def n_starts(self) -> int:
        return len(self.quat) * len(self.trans)

    @property
    def n_searched(self) -> int:
        """Searched starts: every rigid start and its torsion restarts, (1 + R) Q T."""
        return self.n_starts * (1 + self.restarts)


def quaternions(n: int) -> np.ndarray:
    q = np.zeros((n, 4), dtype=np.float32)
    _load().gen_quaternions(n, _ptr(q, ctypes.c_float))
    return q


def translations(n: int, radius: float, center, seed: int = BASE_SEED) -> np.ndarray:
    t = np.zeros((n, 3), dtype=np.float32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    _load().gen_translations(seed, STREAMS["search"], n, radius, _ptr(c, ctypes.c_double), _ptr(t, ctypes.c_float))
    return t


def restart_steps(n_restarts: int, n_steps: int, seed: int = BASE_SEED) -> np.ndarray:
    """Seeded initial torsion turns of the restarts: int32 [n_restarts][16], uniform in [0, n_steps)."""
    rng = np.random.default_rng([seed, 0x7e57a7, n_steps])
    return rng.integers(0, n_steps, (n_restarts, 16)).astype(np.int32)


def make_search(n_quat: int, n_trans: int, n_steps: int, radius: float, center) -> Search:
    return Search(quaternions(n_quat), translations(n_trans, radius, center), int(n_steps))


# ----------------------------------------------------------------------------------------------
# Published benchmark configurations
# ----------------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    pockets: list
    search: Search
    dist: LibDist
    n_lig: int
    n_types: int
    extra: dict = field(default_factory=dict)

    def ligands(self, n_lig: int | None = None, first_id: int = 0, stream: str = "lib") -> Ligands:
        return make_ligands(self.n_lig if n_lig is None else n_lig, self.dist, self.n_types, stream, first_id)


def workload(name: str) -> Workload:
    """The benchmark workloads, named by their sizes."""
    if name == "pocket48-lib100":
        p = make_pocket(48, 8)
        return Workload("pocket48-lib100: 48^3 x 8-type grid, 100 ligands of 24 atoms with 4 rotatable bonds; "
                        "64 quaternions x 8 translations, 64 torsion steps", [p],
                        make_search(64, 8, 64, 2.0, p.center), DIST_FIXED24, 100, 8)
    if name == "pocket96-lib100k":
        p = make_pocket(96, 16)
        return Workload("pocket96-lib100k: 96^3 x 16-type grid, 100k ligands n~N(35,10) in [15,70], "
                        "B~Poisson(5) in [0,12]; 256 quaternions x 32 translations, 256 torsion steps", [p],
                        make_search(256, 32, 256, 4.0, p.center), DIST_DRUGLIKE, 100_000, 16)
    if name == "pockets4-lib250k":
        ps = [make_pocket(d, 16, pocket_id=i) for i, d in enumerate((64, 80, 96, 128))]
        return Workload("pockets4-lib250k: 64^3, 80^3, 96^3 and 128^3 x 16-type grids, 250k ligands of which 5% "
                        "have 80-120 atoms; 256 x 32 starts, 256 steps; top-1000 per pocket", ps,
                        make_search(256, 32, 256, 4.0, ps[0].center), DIST_HEAVY_TAIL, 250_000, 16,
                        {"top_k": 1000})
    raise ValueError(f"unknown workload {name!r}")


def mlp_init(d_in: int = 512, h1: int = 1024, h2: int = 1024, seed: int = BASE_SEED) -> np.ndarray:
    """Seeded initial master weights of the pre-filter network, flat FP32 in the order
    W1 [h1, d_in], b1, W2 [h2, h1], b2, w3 [h2], b3: weights uniform in +-sqrt(6 / fan_in)
    (Kaiming-uniform for ReLU layers; +-sqrt(3 / fan_in) for the linear output), biases zero."""
    rng = np.random.default_rng([seed, 0x6D6C70])
    W1 = rng.uniform(-1, 1, (h1, d_in)) * np.sqrt(6.0 / d_in)
    W2 = rng.uniform(-1, 1, (h2, h1)) * np.sqrt(6.0 / h1)
    w3 = rng.uniform(-1, 1, h2) * np.sqrt(3.0 / h2)
    return np.concatenate([W1.ravel(), np.zeros(h1), W2.ravel(), np.zeros(h2), w3, np.zeros(1)]).astype(np.float32)


def search_for(pocket: Pocket, base: Search, radius: float = 4.0) -> Search:
    """The same search centred on another pocket (translations follow the pocket centre)."""
    return Search(base.quat, translations(len(base.trans), radius, pocket.center), base.n_steps,
                  base.clash_cut, base.clash_w, base.sweep_top, base.passes, base.restarts, base.init_steps)
