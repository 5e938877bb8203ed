"""The C code of the FP64 oracle and of the seeded input generator, and the host code of the HIP
library, under AddressSanitizer and UndefinedBehaviorSanitizer.

Both libraries are rebuilt with -fsanitize=address,undefined into a temporary directory.  A child
Python process with the ASan runtime preloaded then drives every oracle entry point on small seeded
inputs: grids, lookups inside and outside the box in both boundary modes, topology and status of
ligands that the checks reject, the greedy search with start selection and several passes, replay,
brute force, pose filtering and rescoring.  The HIP library is rebuilt with the sanitizers on its
host code only (device code is not instrumented) and runs the C ABI's argument checks and size
queries, which return before any GPU work.  Any sanitizer report fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

DRIVER = r"""
import math, sys
import numpy as np
sys.path.insert(0, sys.argv[3])
import oracle
from paper_2304_09953_amd import inputs as I
oracle.LIB_PATH, I.LIB_PATH = sys.argv[1], sys.argv[2]

def chain(n, rot_bonds):
    xyz = np.array([[i * 1.5 * math.cos(math.pi / 6), (i % 2) * 0.75, 0.0] for i in range(n)])
    bonds = [(i, i + 1) for i in range(n - 1)]
    return xyz, np.zeros(n, np.uint8), bonds, [1 if b in rot_bonds else 0 for b in bonds]

pocket = I.make_pocket((22, 20, 18), 4, n_prot=120, pocket_id=7)
G = oracle.build_grids(pocket)
rng = np.random.default_rng(3)
X = rng.uniform(-12.0, 12.0, (500, 3)) + pocket.center
types = rng.integers(0, 4, 500)
for periodic in (False, True):
    v = oracle.lookup_points(pocket, G, types, X, periodic=periodic)
    assert np.all(np.isfinite(v))

good = I.make_ligands(10, I.DIST_DRUGLIKE, 4, stream="test")
parts = [good.ligand(i) for i in range(good.n_lig)]
x, t, b, r = chain(5, [])
parts += [chain(129, []), (x, np.array([0, 0, 9, 0, 0], np.uint8), b, r), (x, t, b[:3], r[:3]),
          (x, t, [(0, 1), (1, 2), (2, 3), (3, 7)], r), (x, t, [(0, 1), (1, 2), (0, 1), (3, 4)], r),
          (x, t, b, [1, 0, 0, 0]), chain(20, [(i, i + 1) for i in range(1, 18)]), chain(7, [(2, 3)])]
ligs = I.from_parts(parts, 4)
st = oracle.status(ligs)
assert st[:10].tolist() == [0] * 10 and np.all(st[10:-1] != 0) and st[-1] == 0, st
for l in range(ligs.n_lig):
    oracle.topology(ligs, l)

for periodic in (False, True):
    for top, passes in ((0, 1), (3, 2)):
        srch = I.make_search(4, 2, 16, 3.0, pocket.center)
        srch.sweep_top, srch.passes = top, passes
        res = oracle.dock(pocket, G, ligs, srch, per_start=True, periodic=periodic)
        ok = np.flatnonzero(np.isfinite(res["best"]))
        assert len(ok) == 11, res["best"]
        steps = np.asarray(res["steps"])[ok]
        e = oracle.score_poses(pocket, G, ligs, srch, ok, res["start"][ok], steps, periodic=periodic)
        assert np.all(np.isfinite(e))
        if passes == 1:
            oracle.replay(pocket, G, ligs, srch, ok, res["start"][ok], steps, periodic=periodic)
        oracle.greedy_starts(pocket, G, ligs, srch, ok, np.zeros(len(ok), np.int32), periodic=periodic)

srch = I.make_search(2, 2, 8, 3.0, pocket.center)
oracle.exhaustive(pocket, G, ligs, srch, ligs.n_lig - 1)
l = 0
starts = np.array([0, 3, -1, 1, 2, 3], np.int32)  # -1: an absent pose
steps = rng.integers(0, 8, (6, 16)).astype(np.int32)
oracle.filter_rescore(pocket, ligs, srch, l, starts, steps, 1.0)
for bad in (lambda: oracle.filter_rescore(pocket, ligs, srch, l, np.array([4], np.int32), steps[:1], 1.0),
            lambda: oracle.score_poses(pocket, G, ligs, srch, [0], [7], steps[:1]),
            lambda: oracle.pose_coords(ligs, srch, ligs.n_lig, 0)):
    try:
        bad()
        raise AssertionError("an index outside the library or start set was accepted")
    except ValueError:
        pass
oracle.rescore_conformer(pocket, ligs, srch, l, oracle.pose_coords(ligs, srch, l, 1, steps[1]))
print("sanitized oracle ok")
"""


def _gcc(src, out):
    cmd = ["gcc", *SAN, "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-shared", "-fPIC", "-o", out, src, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_oracle_and_generator_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    orc, gen = str(tmp_path / "liboracle_san.so"), str(tmp_path / "libinputs_san.so")
    _gcc(os.path.join(ROOT, "oracle", "dock_oracle.c"), orc)
    _gcc(os.path.join(ROOT, "paper_2304_09953_amd", "inputs", "gen.c"), gen)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", DRIVER, orc, gen, ROOT], capture_output=True, text=True, env=env,
                       timeout=600)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized oracle ok" in r.stdout


ABI_DRIVER = r"""
import sys
sys.path.insert(0, sys.argv[2])
sys.path.insert(0, sys.argv[2] + "/tests")
import paper_2304_09953_amd.dock as d
d.LIB_PATH = sys.argv[1]
import test_abi_cpu as T
for name in ("test_header_declares_the_abi", "test_library_exports_every_declared_symbol",
             "test_calib_argument_errors", "test_surrogate_argument_errors", "test_error_strings",
             "test_grid_desc_validation", "test_size_queries_and_argument_errors"):
    getattr(T, name)()
print("sanitized host library ok")
"""


def test_host_library_under_asan_and_ubsan(tmp_path):
    from paper_2304_09953_amd import build as B
    rt = subprocess.run([B.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    out = str(tmp_path / "libligate_san.so")
    srcs = sorted(os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith(".hip"))
    flags = [f for f in B.HIP_FLAGS if f != "-O3"]
    # the sanitizers instrument the host pass only
    san = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    r = subprocess.run([B.HIPCC, *flags, *san, "-o", out, *srcs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sys.executable, "-c", ABI_DRIVER, out, ROOT], capture_output=True, text=True, env=env,
                       timeout=600)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized host library ok" in r.stdout
