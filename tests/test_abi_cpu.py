"""The C ABI library loads, exports every declared symbol, and rejects bad arguments on the host.

No GPU is needed: argument validation and size queries return before any HIP call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("ligate_dock.h", "ligate_surrogate.h", "ligate_calib.h")]


def _lib():
    from paper_2304_09953_amd import build
    if not os.path.exists(build.LIB_PATH):
        build.build_library()
    from paper_2304_09953_amd import dock
    return dock, dock.load()


def declared_functions(prefix="dock_"):
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(" + prefix + r"\w+)\s*\(", text, re.M)))


def test_every_header_is_covered():
    import glob
    assert sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))) == sorted(HEADERS)


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("dock_build_grids", "dock_pack_ligands", "dock_screen", "dock_topk", "dock_grid_bytes",
              "dock_score_poses", "dock_error_string", "dock_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    dock, lib = _lib()
    from paper_2304_09953_amd import surrogate
    for name in declared_functions("dock_") + declared_functions("surr_") + declared_functions("calib_"):
        assert hasattr(lib, name), name
    assert set(dock.EXPORTS) == set(declared_functions("dock_"))
    assert set(surrogate.SURR_EXPORTS) == set(declared_functions("surr_"))
    assert set(dock.CALIB_EXPORTS) == set(declared_functions("calib_"))
    # nothing else is declared: every function of every header carries one of the three prefixes
    text = "".join(open(h).read() for h in HEADERS)
    all_decl = set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\([^;]*\);", text, re.M | re.S))
    assert all_decl == set(declared_functions("dock_") + declared_functions("surr_") + declared_functions("calib_"))


def test_calib_argument_errors():
    dock, _ = _lib()
    lib = dock._calib_lib()
    assert lib.calib_fma_f32(0, 10, ctypes.c_void_p(16), None) == -1
    assert lib.calib_fma_f32(10, 10, None, None) == -1
    assert lib.calib_cache_read(ctypes.c_void_p(16), 16384 + 4096, 1, 1, ctypes.c_void_p(16), None) == -1
    assert lib.calib_cache_read(ctypes.c_void_p(8), 16384, 1, 1, ctypes.c_void_p(16), None) == -1
    assert lib.calib_cache_read(ctypes.c_void_p(16), 16384, 0, 1, ctypes.c_void_p(16), None) == -1


def test_surrogate_argument_errors():
    _, lib = _lib()
    from paper_2304_09953_amd import surrogate as SG
    lib = SG._lib()
    nm, nb = ctypes.c_int64(), ctypes.c_int64()
    assert lib.surr_param_count(512, 1024, 1024, ctypes.byref(nm), ctypes.byref(nb)) == 0
    assert nm.value == 1024 * 512 + 1024 + 1024 * 1024 + 1024 + 1024 + 1
    assert nb.value == 1024 * 512 + 1024 * 1024 + 1024
    bad = SG.SurrModel(500, 1024, 1024, 1, 1, 1, 1, 1)
    sz = ctypes.c_size_t()
    assert lib.surr_forward(ctypes.byref(bad), None, 8, None, None, ctypes.byref(sz), None) == -1
    good = SG.SurrModel(512, 1024, 1024, 1, 1, 1, 1, 1)
    assert lib.surr_forward(ctypes.byref(good), None, 8, None, None, ctypes.byref(sz), None) == 0
    assert lib.surr_backward(ctypes.byref(good), None, None, 30, None, None, ctypes.byref(sz), None) == -1
    assert lib.surr_features(None, None, None, None, 5, 10, 17, None, None, None, None, None) == -2
    fake = ctypes.c_void_p(0x1000)
    assert lib.surr_average(fake, 0, 10, fake, None) == -1
    assert lib.surr_average(fake, 65, 10, fake, None) == -1
    assert lib.surr_average(None, 4, 10, fake, None) == -1
    assert lib.surr_average(None, 4, 0, None, None) == 0


def test_error_strings():
    dock, lib = _lib()
    assert lib.dock_error_string(0) == b"ok"
    assert b"workspace" in lib.dock_error_string(-4)


def _desc(dock, **kw):
    d = dict(nx=8, ny=9, nz=10, n_types=4, origin=(ctypes.c_float * 3)(0, 0, 0), spacing=0.375, layout=0,
             boundary=0, w_out=10.0)
    d.update(kw)
    return dock.GridDesc(**d)


def test_grid_desc_validation():
    dock, lib = _lib()
    out = ctypes.c_size_t()
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock)), ctypes.byref(out)) == 0
    assert out.value == 4 * 4 * 8 * 9 * 10
    for bad in (dict(nx=1), dict(spacing=0.0), dict(layout=3), dict(boundary=7)):
        assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, **bad)), ctypes.byref(out)) == -1
        assert lib.dock_last_error() != b""
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, n_types=33)), ctypes.byref(out)) == -2
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, nx=300, ny=300, nz=300)), ctypes.byref(out)) == -2
    # xy4 layout: 16-byte records in 128-byte bricks of 2 x 2 x 2, dims rounded up to even;
    # all type grids below 2^31 bytes, one type grid below 2^28
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=1)), ctypes.byref(out)) == 0
    assert out.value == 128 * (4 * 5 * 5) * 4
    odd = dict(nx=255, ny=255, nz=255, n_types=1)  # < 2^24 nodes, but 128^3 bricks = 2^28 bytes
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=0, **odd)), ctypes.byref(out)) == 0
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=1, **odd)), ctypes.byref(out)) == -2
    # xy4 record offsets use 24-bit multiplies: (nx rounded up to even) * ceil(ny / 2) <= 2^18
    wide = dict(nx=2048, ny=1024, nz=2, n_types=1)  # 2048 * 512 = 2^20
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=0, **wide)), ctypes.byref(out)) == 0
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=1, **wide)), ctypes.byref(out)) == -2
    edge = dict(nx=1024, ny=512, nz=4, n_types=1)  # 1024 * 256 = 2^18
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=1, **edge)), ctypes.byref(out)) == 0
    big = dict(nx=200, ny=200, nz=200, n_types=17)  # 8e6 nodes x 17 types x 16 B > 2^31
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=0, **big)), ctypes.byref(out)) == 0
    assert lib.dock_grid_bytes(ctypes.byref(_desc(dock, layout=1, **big)), ctypes.byref(out)) == -2


def test_size_queries_and_argument_errors():
    dock, lib = _lib()
    sz = ctypes.c_size_t()
    assert lib.dock_pack_ligands(None, None, None, None, None, None, 10, 300, 16, None, ctypes.byref(sz), None,
                                 None) == 0
    assert sz.value > 300 * 12
    assert lib.dock_pack_ligands(None, None, None, None, None, None, -1, 300, 16, None, ctypes.byref(sz), None,
                                 None) == -1
    assert lib.dock_pack_ligands(None, None, None, None, None, None, 10, 300, 40, None, ctypes.byref(sz), None,
                                 None) == -2
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: size queries return before any device work
    s = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0)
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(s), None, None, None, None,
                           None, None, None, ctypes.byref(sz), None) == 0
    assert sz.value > 0
    s_bad = dock.SearchDesc(4, fake, 2, fake, 2048, 2.5, 10.0, 0, 0)
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(s_bad), None, None, None, None,
                           None, None, None, ctypes.byref(sz), None) == -2
    # search budget: the selection adds n_lig x K start ids to the workspace; bad fields are refused
    base = sz.value
    s_top = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0, 3, 2)
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(s_top), None, None, None, None,
                           None, None, None, ctypes.byref(sz), None) == 0
    assert sz.value >= base + 10 * 3 * 4
    for top, passes, code in ((-1, 1, -1), (0, -1, -1), (0, 17, -1), (4, 1, 0), (8, 16, 0)):
        sb = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0, top, passes)
        assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(sb), None, None, None,
                               None, None, None, None, ctypes.byref(sz), None) == code, (top, passes)
    many = dock.SearchDesc(4096, fake, 4, fake, 64, 2.5, 10.0, 0, 0, 100, 1)  # 16384 starts to rank
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(many), None, None, None, None,
                           None, None, None, ctypes.byref(sz), None) == -2
    all_of_many = dock.SearchDesc(4096, fake, 4, fake, 64, 2.5, 10.0, 0, 0, 16384, 1)  # nothing to select
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(all_of_many), None, None,
                           None, None, None, None, None, ctypes.byref(sz), None) == 0
    # torsion restarts: at most DOCK_MAX_RESTARTS, need the initial-turn table, not with sweep_top
    for R, init, top, code in ((2, fake, 0, 0), (64, fake, 0, 0), (65, fake, 0, -1), (-1, fake, 0, -1),
                               (2, None, 0, -1), (2, fake, 5, -1)):
        sr = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0, top, 1, R, init)
        assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, 10, 300, ctypes.byref(sr), None, None, None,
                               None, None, None, None, ctypes.byref(sz), None) == code, (R, init, top)
    assert "DOCK_MAX_RESTARTS 64" in open(os.path.join(ROOT, "include", "ligate_dock.h")).read()
    # the allocation-free screen refuses, before any HIP call, a screen whose scratch exceeds its array
    assert "#define DOCK_NOALLOC_SCRATCH_BYTES (32u << 20)" in open(os.path.join(ROOT, "include", "ligate_dock.h")).read()
    big = 2_000_000  # about 25 bytes of scratch per ligand: 50 MB > 32 MiB
    assert lib.dock_screen(ctypes.byref(_desc(dock)), None, None, big, 300, ctypes.byref(s), None, None, None, None,
                           None, None, None, ctypes.byref(sz), None) == 0
    assert sz.value > (32 << 20)
    assert lib.dock_screen_noalloc(ctypes.byref(_desc(dock)), fake, fake, big, 300, ctypes.byref(s), fake, fake, fake,
                                   None, None, None, None) == -2
    assert b"scratch" in lib.dock_last_error()
    sel_big = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0, 3, 1)
    assert lib.dock_screen_noalloc(ctypes.byref(_desc(dock)), fake, fake, 10, 300, ctypes.byref(s_bad), fake, fake,
                                   fake, None, None, None, None) == -2  # the screen's own limits come first
    assert lib.dock_screen_noalloc(ctypes.byref(_desc(dock)), None, fake, 10, 300, ctypes.byref(sel_big), fake, fake,
                                   fake, None, None, None, None) == -1
    # dock_rescore checks every argument, the type table included, before its first launch
    T = 4
    params = (dock.TypeParam * T)(*[dock.TypeParam(1.5, 0.1 if t < T - 1 else -0.1, 0.0) for t in range(T)])
    pot = dock.Potential(10.0, 0.5, 83.0)
    s8 = dock.SearchDesc(4, fake, 2, fake, 64, 2.5, 10.0, 0, 0)
    assert lib.dock_rescore(ctypes.byref(_desc(dock)), fake, fake, 10, 300, ctypes.byref(s8), fake, fake, fake, 30,
                            params, ctypes.byref(pot), 4, 1.0, fake, fake, fake, fake, fake, fake, None, None) == -1
    assert b"eps of type 3" in lib.dock_last_error()
    assert lib.dock_merge_pockets(fake, 0, 10, fake, fake, None) == -1
    assert lib.dock_merge_pockets(fake, 2, 0, fake, fake, None) == -1
    assert lib.dock_merge_pockets(None, 2, 10, fake, fake, None) == -1
    assert lib.dock_topk(None, None, 100, 10, None, None, None, ctypes.byref(sz), None) == 0
    assert lib.dock_topk(None, None, 100, 101, None, None, None, ctypes.byref(sz), None) == -1
    assert lib.dock_topk(None, None, 0, 1, None, None, None, ctypes.byref(sz), None) == -1
    # a workspace smaller than the query is refused before anything is enqueued
    small = ctypes.c_size_t(16)
    assert lib.dock_topk(fake, None, 100, 10, fake, fake, fake, ctypes.byref(small), None) == -4


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2304_09953_amd import dock
    monkeypatch.setattr(dock, "_lib", None)
    monkeypatch.setattr(dock, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(dock.DockError):
        dock.load()
