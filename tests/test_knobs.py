"""The knob tuner's host logic on a synthetic objective with a known constrained optimum."""
import numpy as np
import pytest

from paper_2304_09953_amd import knobs as K


def _synthetic(cfg):
    # cost grows with the work; recall saturates with the work, more with passes, restarts and every start
    work = cfg["n_quat"] * cfg["n_trans"] * cfg["n_steps"] / (32 * 8 * 64)
    swept = 1.0 if cfg["sweep_top"] == 0 else min(1.0, cfg["sweep_top"] / (cfg["n_quat"] * cfg["n_trans"]))
    r = cfg.get("restarts", 0)
    cost = work * (0.1 + 0.9 * swept) * cfg["passes"] ** 0.8 * (1 + r)
    reach = 1.0 - 0.08 * (cfg.get("radius", 4.0) - 4.0) ** 2  # the translations cover the site best at 4 A
    recall = 1 - np.exp(-0.9 * np.log2(max(work * 2, 1.01)) * (0.5 + 0.5 * swept) * (1 + 0.15 * (cfg["passes"] - 1))
                        * (1 + 0.1 * r) * reach)
    return cost, recall


def test_grid_collapses_selection_and_excludes_restarts_with_it():
    g = K.grid()
    assert len(g) == len({tuple(c.values()) for c in g})
    assert all(c["sweep_top"] < c["n_quat"] * c["n_trans"] for c in g)
    assert not any(c["sweep_top"] and c["restarts"] for c in g)  # restarts only over every start
    assert any(c["restarts"] for c in g)
    X = K.encode(g)
    assert X.shape == (len(g), len(K.SPACE)) and X.min() >= 0 and X.max() <= 1


def test_gp_interpolates_its_data():
    rng = np.random.default_rng(0)
    X = rng.random((12, 3))
    y = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    m, s = K.GP(length=0.5, noise=1e-8).fit(X, y).predict(X)
    assert np.allclose(m, y, atol=1e-4) and np.all(s < 1e-2)


def test_space_is_too_large_to_enumerate_by_screens():
    g = K.grid()
    assert len(g) >= 10_000
    assert len(K.grid(K.SMALL_SPACE)) == 390
    X = K.encode(g)
    r = X[:, list(K.SPACE).index("radius")]
    assert r.min() == 0.0 and r.max() == 1.0 and len(np.unique(r)) == 4  # linear axis


@pytest.mark.parametrize("space", ["small", "wide"])
def test_optimizer_finds_the_constrained_optimum(space):
    target = 0.9
    sp = K.SMALL_SPACE if space == "small" else K.SPACE
    truth = K.best_feasible([{"cfg": c, "cost": _synthetic(c)[0], "recall": _synthetic(c)[1]} for c in K.grid(sp)],
                            target)
    calls = []
    res = K.optimize(lambda c: calls.append(c) or _synthetic(c), target, space=sp, n_init=6, n_iter=24, seed=1)
    assert len(calls) == 30 and len(K.grid(sp)) > 150
    best = res["best"]
    assert best is not None and best["recall"] >= target
    assert best["cost"] <= (1.10 if space == "small" else 1.5) * truth["cost"]
    # and on average it does better than random search with the same number of screens
    rnd = [K.random_search(_synthetic, target, 30, space=sp, seed=s)["best"] for s in range(8)]
    rnd_cost = np.mean([r["cost"] if r else np.inf for r in rnd])
    assert best["cost"] <= rnd_cost
