"""Writes tiny_screen.json: the oracle's results on a tiny seeded docking case (a regression fixture).

The paper describes the screening workflow in words (§2; the batched redesign in §3.3) and prints no
worked example of the computation, so no value here is taken from it.  This script calls only the
oracle and the seeded input generator.  tests/test_golden.py recomputes the same quantities and
compares them with the file, so that any change to the oracle's arithmetic shows up, and has to be
justified by the passage or reading behind it before the fixture is rewritten by running this script:

    python tests/golden/make_golden.py      (from the repository root)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2304_09953_amd import inputs as I  # noqa: E402

PATH = os.path.join(HERE, "tiny_screen.json")


def case():
    """The tiny case: a 32^3 pocket with 4 atom types and 80 protein atoms, five ligands of 5-11 atoms with
    up to four rotatable bonds, 16 quaternions x 2 translations, 16 torsion steps."""
    pocket = I.make_pocket(32, 4, n_prot=80, pocket_id=21)
    dist = I.LibDist(n_mean=8.0, n_sd=2.0, n_min=5, n_max=11, b_mean=2.0, b_min=0, b_max=4, offset_range=2.0)
    ligs = I.make_ligands(5, dist, 4, stream="tiny")
    srch = I.make_search(16, 2, 16, 1.0, pocket.center)
    return pocket, ligs, srch


def compute():
    """Every quantity the fixture records, from the oracle."""
    pocket, ligs, srch = case()
    G = oracle.build_grids(pocket)
    rng = np.random.default_rng(21)
    nodes = np.stack([rng.integers(0, n, 40) for n in G.shape], 1)
    # points inside the box and some outside it (clamp and restraint)
    lo = pocket.origin.astype(np.float64)
    hi = lo + pocket.spacing * (np.array(pocket.dims) - 1)
    pts = lo - 1.0 + rng.random((12, 3)) * (hi - lo + 2.0)
    types = rng.integers(0, pocket.n_types, 12)
    res = oracle.dock(pocket, G, ligs, srch, per_start=True)
    B = ligs.n_rot
    top_s, top_i = oracle.topk(res["best"], 3, ligs.ids)
    poses_l = np.array([0, 1, 2, 3, 4, 4], np.int64)
    poses_p = np.array([0, 5, 9, 15, 3, 3], np.int32)
    poses_s = np.zeros((6, 16), np.int32)
    poses_s[4, :4] = [1, 2, 3, 4]
    poses_s[5, :4] = [15, 0, 8, 7]
    return {
        "grid_nodes": nodes.tolist(),
        "grid_values": [float(G[tuple(n)]) for n in nodes],
        "lookup_points": pts.tolist(), "lookup_types": types.tolist(),
        "lookup_values": oracle.lookup_points(pocket, G, types, pts).tolist(),
        "status": oracle.status(ligs).tolist(),
        "n_rot": B.tolist(),
        "best": res["best"].tolist(),
        "best_start": res["start"].tolist(),
        "best_steps": [res["steps"][i][:B[i]].tolist() for i in range(ligs.n_lig)],
        "start_finals": res["finals"].tolist(),
        "topk_scores": np.asarray(top_s).tolist(), "topk_ids": np.asarray(top_i).tolist(),
        "pose_lig": poses_l.tolist(), "pose_start": poses_p.tolist(), "pose_steps": poses_s.tolist(),
        "pose_scores": oracle.score_poses(pocket, G, ligs, srch, poses_l, poses_p, poses_s).tolist(),
    }


if __name__ == "__main__":
    out = {"what": "the oracle's results on the tiny seeded case of tests/golden/make_golden.py",
           "cites": {"best pose per ligand, library ranked by it": "paper §2",
                     "multi-start search, batched screening": "paper §2, §3.3",
                     "every formula": "the readings of the paper listed with the oracle"},
           **compute()}
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", PATH)
