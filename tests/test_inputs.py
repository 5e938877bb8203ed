"""The seeded input generator: determinism, validity and the configured distributions."""
import numpy as np

import oracle
from paper_2304_09953_amd import inputs as I


def test_ligand_is_independent_of_chunking():
    a = I.make_ligands(50, I.DIST_DRUGLIKE, 16, first_id=1000)
    b = I.make_ligands(20, I.DIST_DRUGLIKE, 16, first_id=1030)
    for j in range(20):
        xa, ta, ba, ra = a.ligand(30 + j)
        xb, tb, bb, rb = b.ligand(j)
        assert np.array_equal(xa, xb) and np.array_equal(ta, tb)
        assert np.array_equal(ba, bb) and np.array_equal(ra, rb)
    c = I.make_ligands(50, I.DIST_DRUGLIKE, 16, first_id=1000, stream="train")
    assert not np.array_equal(a.xyz[:100], c.xyz[:100])


def test_generated_trees_are_valid_and_clash_free():
    ligs = I.make_ligands(300, I.DIST_HEAVY_TAIL, 16, stream="test")
    assert np.all(oracle.status(ligs) == 0)
    for l in range(0, 300, 7):
        x, t, b, r = ligs.ligand(l)
        x = x.astype(np.float64)
        bl = np.linalg.norm(x[b[:, 0]] - x[b[:, 1]], axis=1)
        assert np.allclose(bl, 1.5, atol=1e-5)
        topo = oracle.topology(ligs, l)
        if len(topo["pairs"]):
            d = np.linalg.norm(x[topo["pairs"][:, 0]] - x[topo["pairs"][:, 1]], axis=1)
            assert d.min() >= 2.6 - 1e-5
        assert np.all(t < 16)


def test_library_distributions():
    l2 = I.make_ligands(20000, I.DIST_DRUGLIKE, 16)
    n, b = l2.n_atoms, l2.n_rot
    assert n.min() >= 15 and n.max() <= 70 and abs(n.mean() - 35.0) < 0.3
    assert b.min() >= 0 and b.max() <= 12 and abs(b.mean() - 5.0) < 0.15
    l3 = I.make_ligands(20000, I.DIST_HEAVY_TAIL, 16)
    heavy = l3.n_atoms >= 80
    assert abs(heavy.mean() - 0.05) < 0.006 and l3.n_atoms.max() <= 120
    l1 = I.make_ligands(100, I.DIST_FIXED24, 8)
    assert np.all(l1.n_atoms == 24) and np.all(l1.n_rot == 4)
    # type weights proportional to 1/(1+t)
    w = 1.0 / (1.0 + np.arange(16))
    freq = np.bincount(l2.types, minlength=16) / len(l2.types)
    assert np.allclose(freq, w / w.sum(), atol=0.003)


def test_search_sets_and_pocket_frame():
    q = I.quaternions(256)
    assert np.allclose(np.linalg.norm(q.astype(np.float64), axis=1), 1.0, atol=1e-6)
    # near-uniform over rotations: |<q_i, q_j>| is never close to 1 for i != j
    G = np.abs(q.astype(np.float64) @ q.T.astype(np.float64))
    np.fill_diagonal(G, 0)
    assert G.max() < 0.99
    p = I.make_pocket(96, 16)
    assert np.all(p.origin * 8 == np.round(p.origin * 8))
    t = I.translations(32, 4.0, p.center)
    assert np.array_equal(t[0], p.center.astype(np.float32))
    assert np.all(np.linalg.norm(t - p.center, axis=1) <= 4.0 + 1e-5)
    r = np.linalg.norm(p.prot_xyz - p.center, axis=1)
    assert r.min() >= 6.0 - 1e-4 and r.max() <= 12.0 + 1e-4 and len(r) == 300
