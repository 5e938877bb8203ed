"""The allocation-free screen entry point (dock_screen_noalloc) against dock_screen.

Both enqueue the same kernels; only where the scratch lives differs, so every output must be
equal bit for bit.  Two calls in a row, the second on a smaller library with start selection and
two passes, show that nothing left in the shared device scratch by one call leaks into the next.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2304_09953_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_noalloc_screen_equals_dock_screen():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09953_amd import dock
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket48-lib100")
    dp = P.DevicePocket(W.pockets[0])
    big = W.ligands()
    small = big.subset(np.arange(0, 100, 7))
    cases = [(big, W.search), (small, dataclasses.replace(W.search, sweep_top=32, passes=2))]
    for ligs, srch in cases:
        say(f"dock_screen_noalloc: {ligs.n_lig} ligands, sweep_top {srch.sweep_top}, passes {srch.passes}")
        lib = P.DeviceLibrary(ligs)
        ds = P.DeviceSearch(srch)
        ref = P.screen(dp, lib, ds, start_scores=True)
        n, N = ligs.n_lig, srch.n_searched
        dev = dp.grids.device
        out = dict(best_score=torch.full((n,), -7.0, device=dev), best_start=torch.full((n,), -7, dtype=torch.int32,
                                                                                        device=dev),
                   best_steps=torch.full((n * 16,), -7, dtype=torch.int16, device=dev),
                   start_scores=torch.full((n * N,), -7.0, device=dev),
                   start_steps=torch.full((n * N * 16,), -7, dtype=torch.int16, device=dev),
                   pose_count=torch.full((1,), -7, dtype=torch.int64, device=dev))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        dock.screen_noalloc(dp.desc, dp.grids, lib.pack, n, lib.n_atoms, ds.desc, out["best_score"], out["best_start"],
                            out["best_steps"], out["start_scores"], out["pose_count"], None, out["start_steps"])
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(out["best_score"], ref.best_score)
        assert torch.equal(out["best_start"], ref.best_start)
        assert torch.equal(out["best_steps"], ref.best_steps.reshape(-1))
        assert torch.equal(out["start_scores"], ref.start_scores)
        # steps are defined for searched starts only (with sweep_top the others are not written)
        searched = torch.isfinite(ref.start_scores).repeat_interleave(16)
        assert torch.equal(out["start_steps"][searched], ref.start_steps[searched])
        assert bool(torch.all(out["start_steps"][~searched] == -7))
        assert torch.equal(out["pose_count"], ref.pose_count)
        assert np.isfinite(out["best_score"].cpu().numpy()).all()
