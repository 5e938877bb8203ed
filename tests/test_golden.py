"""The oracle against its stored results on a tiny seeded case (tests/golden/tiny_screen.json, written by
tests/golden/make_golden.py from the oracle alone).  Integers must match exactly and floating-point
values to 1e-12 relative: the oracle is deterministic FP64, so any difference is a change of its
arithmetic, which must name the passage or reading behind it before the fixture is rewritten."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def test_oracle_reproduces_its_stored_tiny_screen():
    want = json.load(open(make_golden.PATH))
    got = make_golden.compute()
    assert set(got) <= set(want)
    for key, val in got.items():
        a = np.asarray(val, dtype=object if key == "best_steps" else None)
        b = np.asarray(want[key], dtype=object if key == "best_steps" else None)
        if key == "best_steps":
            assert [list(x) for x in a] == [list(x) for x in b], key
        elif np.issubdtype(np.asarray(val).dtype, np.integer):
            assert np.array_equal(a, b), key
        else:
            a, b = np.asarray(val, np.float64), np.asarray(want[key], np.float64)
            assert a.shape == b.shape, key
            assert np.all((a == b) | (np.abs(a - b) <= 1e-12 * np.maximum(1.0, np.abs(b)))), key
