"""Property tests of the FP64 oracle on random small inputs drawn by Hypothesis (derandomized, so
every run draws the same examples).

* Torsion moves are rigid within each fragment: every bond length and every distance between two
  atoms that no rotatable bond separates is that of the reference conformer, for any steps.
* The greedy search never raises a start's score: every sweep offers step 0 (no turn), and the
  argmin takes the lowest score with ties to the lowest step.
* Trilinear interpolation reproduces any affine field exactly inside the box.
* Top-k is the first k of a sort by (score, id) with NaN as +inf, whatever ties, NaNs or signed
  zeros the scores hold.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2304_09953_amd import inputs as I

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@st.composite
def trees(draw, max_n=20, n_types=4):
    """A tree of degree <= 4 with 1.5 A bonds in random directions and random rotatable bonds."""
    n = draw(st.integers(3, max_n))
    deg = [1] + [1] * (n - 1)
    deg[0] = 0
    parent = [-1]
    for i in range(1, n):
        j = draw(st.sampled_from([a for a in range(i) if deg[a] < 4]))
        parent.append(j)
        deg[j] += 1
    rng = np.random.default_rng(draw(st.integers(0, 2**32 - 1)))
    xyz = np.zeros((n, 3))
    for i in range(1, n):
        v = rng.normal(size=3)
        xyz[i] = xyz[parent[i]] + 1.5 * v / np.linalg.norm(v)
    bonds = [(parent[i], i) for i in range(1, n)]
    eligible = [deg[a] >= 2 and deg[b] >= 2 for a, b in bonds]  # terminal bonds cannot rotate
    rot = [int(e and draw(st.booleans())) for e in eligible]
    while sum(rot) > 16:
        rot[rot.index(1)] = 0
    types = rng.integers(0, n_types, n).astype(np.uint8)
    return xyz, types, bonds, rot


def _fragments(n, bonds, rot):
    """Component label of every atom after cutting the rotatable bonds (union-find)."""
    lab = list(range(n))

    def find(a):
        while lab[a] != a:
            lab[a] = lab[lab[a]]
            a = lab[a]
        return a
    for (a, b), r in zip(bonds, rot):
        if not r:
            lab[find(a)] = find(b)
    return np.array([find(a) for a in range(n)])


@pytest.fixture(scope="module")
def field():
    pocket = I.make_pocket(24, 4, n_prot=80, pocket_id=9)
    return pocket, oracle.build_grids(pocket)


@SETTINGS
@given(tree=trees(), steps_seed=st.integers(0, 2**32 - 1), start=st.integers(0, 3))
def test_torsion_moves_are_rigid_within_fragments(tree, steps_seed, start):
    xyz, types, bonds, rot = tree
    ligs = I.from_parts([tree], 4)
    assert oracle.status(ligs)[0] == 0
    srch = I.make_search(2, 2, 12, 2.0, np.zeros(3))
    steps = np.random.default_rng(steps_seed).integers(0, 12, 16)
    X = oracle.pose_coords(ligs, srch, 0, start, steps)
    ref = ligs.ligand(0)[0].astype(np.float64)
    d_ref = np.linalg.norm(ref[:, None] - ref[None], axis=-1)
    d = np.linalg.norm(X[:, None] - X[None], axis=-1)
    for a, b in bonds:
        assert abs(d[a, b] - d_ref[a, b]) < 1e-9
    frag = _fragments(len(types), bonds, rot)
    same = frag[:, None] == frag[None, :]
    assert np.all(np.abs(d - d_ref)[same] < 1e-9)


@SETTINGS
@given(tree=trees(), step=st.integers(1, 11), start=st.integers(0, 3), pick=st.integers(0, 15))
def test_a_turn_moves_only_its_moving_side_and_not_its_axis_atoms(tree, step, start, pick):
    # the moving side of torsion a-b holds b, which lies on the axis: a turn leaves a, b and the fixed
    # side where they are, and every moving atom at its distance from a and from b
    xyz, types, bonds, rot = tree
    ligs = I.from_parts([tree], 4)
    tp = oracle.topology(ligs, 0)
    if tp["B"] == 0:
        return
    k = pick % tp["B"]
    srch = I.make_search(2, 2, 12, 2.0, np.zeros(3))
    steps = np.zeros(16, np.int64)
    steps[k] = step
    X0 = oracle.pose_coords(ligs, srch, 0, start, np.zeros(16, np.int64))
    X = oracle.pose_coords(ligs, srch, 0, start, steps)
    a, b, mv = tp["tor_a"][k], tp["tor_b"][k], tp["moving"][k]
    assert mv[b] and not mv[a]
    still = ~mv
    still[b] = True
    assert np.max(np.abs(X[still] - X0[still])) < 1e-9
    for end in (a, b):
        assert np.allclose(np.linalg.norm(X[mv] - X[end], axis=1), np.linalg.norm(X0[mv] - X0[end], axis=1),
                           atol=1e-9)


@SETTINGS
@given(tree=trees(max_n=14))
def test_greedy_never_raises_a_start_score(field, tree):
    pocket, G = field
    ligs = I.from_parts([tree], 4)
    srch = I.make_search(3, 2, 8, 2.0, pocket.center)
    res = oracle.dock(pocket, G, ligs, srch, per_start=True)
    QT = srch.n_starts
    rigid = oracle.score_poses(pocket, G, ligs, srch, np.zeros(QT, np.int64), np.arange(QT), np.zeros((QT, 16)))
    fin = res["finals"][0]
    assert np.all(fin <= rigid + 1e-12 * np.maximum(1.0, np.abs(rigid)))
    assert res["best"][0] == fin.min() and fin[res["start"][0]] == fin.min()


@SETTINGS
@given(coef=st.lists(st.integers(-40, 40).map(lambda v: v / 8.0), min_size=4, max_size=4),
       pts=st.lists(st.tuples(*[st.floats(0, 1)] * 3), min_size=1, max_size=20))
def test_trilinear_reproduces_affine_fields(coef, pts):
    dims = (6, 5, 4)
    R, e, q = I.type_table(1)
    p = I.Pocket(dims, 1, np.array([0.5, -1.0, 2.0], np.float32), 0.5, np.zeros((1, 3), np.float32),
                 np.zeros(1, np.int32), R, e, q)
    kk, jj, ii = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    c0, cx, cy, cz = coef  # multiples of 1/8: the field's node values are exact in FP32
    G = (c0 + cx * ii + cy * jj + cz * kk)[None]
    G32 = G.astype(np.float32)
    assert np.array_equal(G32.astype(np.float64), G)
    u = np.array(pts) * (np.array(dims) - 1)
    x = p.origin.astype(np.float64) + p.spacing * u
    got = oracle.lookup_points(p, G32, np.zeros(len(u)), x)
    want = c0 + cx * u[:, 0] + cy * u[:, 1] + cz * u[:, 2]
    assert np.allclose(got, want, rtol=0, atol=1e-9 * (1 + np.abs(want)))


@SETTINGS
@given(scores=st.lists(st.one_of(st.integers(-3, 3).map(float), st.just(float("nan")), st.just(-0.0),
                                 st.just(float("inf"))), min_size=1, max_size=60),
       k=st.integers(1, 60), seed=st.integers(0, 1000))
def test_topk_is_the_head_of_a_sort(scores, k, seed):
    k = min(k, len(scores))
    ids = np.random.default_rng(seed).permutation(len(scores)) + 100
    got_s, got_i = oracle.topk(scores, k, ids)
    key = [(float("inf") if s != s else s, i) for s, i in zip(scores, ids)]
    ref = sorted(key)[:k]
    assert [i for _, i in ref] == got_i.tolist()
    assert all((a == b) or (a != a and b == float("inf")) for a, (b, _) in zip(got_s.tolist(), ref))
