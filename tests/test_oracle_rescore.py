"""Pins of the oracle's pose filtering and rescoring (the steps after the search): the rescoring
pair energy against the grid's, the per-atom cap, the RMSD filter against rigid translations."""
import numpy as np
import pytest

import oracle
from paper_2304_09953_amd import inputs as I


@pytest.fixture(scope="module")
def pocket():
    return I.make_pocket(32, 4, pocket_id=31)


def test_rescore_pair_equals_the_grid_pair_at_unit_distance(pocket):
    # Coulomb over 4 r^2 and over 4 r agree where r = 1; the 6-12 term is shared
    for a in range(4):
        for b in range(4):
            assert oracle.rescore_pair(pocket, 1.0, a, b) == pytest.approx(oracle.pair_energy(pocket, 1.0, a, b),
                                                                            rel=1e-15, abs=1e-15)


def test_rescore_pair_coulomb_scales_as_inverse_square(pocket):
    # rescore - grid pair = K q_a q_b (1/r^2 - 1/r), K = coulomb_k, q from the type table
    for a, b in ((0, 3), (1, 2), (3, 3)):
        kqq = pocket.coulomb_k * pocket.type_q[a] * pocket.type_q[b]
        for r in (0.7, 2.0, 3.5, 9.0):
            g = oracle.pair_energy(pocket, r, a, b)
            d = oracle.rescore_pair(pocket, r, a, b) - g
            # the difference of two sums dominated by the 6-12 term at short range: rounding of that term
            assert d == pytest.approx(kqq * (1 / r ** 2 - 1 / r), rel=1e-12, abs=1e-14 * max(1.0, abs(g)))
    # r is floored at r_min like the grid's
    assert oracle.rescore_pair(pocket, 0.1, 1, 2) == oracle.rescore_pair(pocket, pocket.r_min, 1, 2)


def test_single_atom_rescore_is_the_capped_pair(pocket):
    one = I.make_pocket(32, 4, n_prot=1, pocket_id=32)
    p = one.prot_xyz[0].astype(np.float64)
    srch = I.make_search(2, 1, 8, 1.0, one.center)
    for t in range(4):
        lig = I.from_parts([(np.zeros((1, 3)), [t], np.zeros((0, 2)), [])], 4)
        for r in (0.9, 3.0, 6.0):
            X = (p + np.array([r, 0.0, 0.0]))[None]
            got = oracle.rescore_conformer(one, lig, srch, 0, X)
            ref = min(one.cap, oracle.rescore_pair(one, r, t, int(one.prot_type[0])))
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)
    assert oracle.rescore_conformer(one, lig, srch, 0, (p + np.array([0.2, 0, 0]))[None]) == one.cap


def test_filter_translations_duplicates_and_rescore(pocket):
    ligs = I.make_ligands(3, I.DIST_DRUGLIKE, 4, stream="test", first_id=900)
    srch = I.make_search(3, 4, 16, 3.0, pocket.center)
    T = len(srch.trans)
    for l in range(ligs.n_lig):
        # poses 0-3: one quaternion, four translations, no turns; pose 4 repeats pose 0; pose 5 turned
        start = np.array([0, 1, 2, 3, 0, 1 * T + 2], np.int32)
        steps = np.zeros((6, 16), np.int32)
        steps[5, :ligs.n_rot[l]] = 3
        for rmin in (0.0, 0.5):
            r = oracle.filter_rescore(pocket, ligs, srch, l, start, steps, rmin)
            # a pose and its translate by d are |d| apart (same atoms, rigid shift)
            d = np.linalg.norm(srch.trans[1].astype(np.float64) - srch.trans[0].astype(np.float64))
            assert r["nearest"][1] == pytest.approx(d, rel=1e-12)
            assert r["kept"][0] and np.isinf(r["nearest"][0])
            assert r["nearest"][4] == 0.0 and r["kept"][4] == (rmin == 0.0)
            for i in np.flatnonzero(r["kept"]):
                X = oracle.pose_coords(ligs, srch, l, int(start[i]), steps[i])
                assert r["rescore"][i] == pytest.approx(oracle.rescore_conformer(pocket, ligs, srch, l, X), rel=1e-12)
            assert np.all(np.isnan(r["rescore"][~r["kept"]]))
        # every translation is at least its distance apart: with a threshold beyond all of them only
        # pose 0 and what is not near it survive
        big = oracle.filter_rescore(pocket, ligs, srch, l, start, steps, 1e6)
        assert big["kept"].tolist() == [True, False, False, False, False, False]
    # an absent pose (start -1) is dropped
    r = oracle.filter_rescore(pocket, ligs, srch, 0, np.array([-1, 0], np.int32), np.zeros((2, 16), np.int32), 1.0)
    assert r["kept"].tolist() == [False, True] and np.isnan(r["rescore"][0]) and np.isinf(r["nearest"][1])
