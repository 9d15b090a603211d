"""The oracle against its stored results on one tiny problem
(tests/golden/oracle_tiny.json, written by tests/golden/make_golden.py from
the oracle alone).  A regression guard for the oracle's arithmetic: any
change to it must be justified against the paper before the file is
rewritten.  Tolerance 1e-12 relative (summation order only)."""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "oracle_tiny.json")) as f:
        return json.load(f)


def close(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    assert a.shape == b.shape
    assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())


def test_oracle_matches_its_stored_results(golden):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    b = np.asarray(golden["b"], np.float32).reshape(golden["b_shape"])
    d = np.asarray(golden["d"], np.float32).reshape(golden["d_shape"])
    b2, d2 = mg.inputs()
    assert np.array_equal(b, b2) and np.array_equal(d, d2)
    got = mg.compute(b, d)
    for key in ("z", "theta", "resid", "d_learned", "mu", "gamma", "objective", "dloss_dd"):
        close(got[key], golden[key])
    close([got["loss"], got["dloss_dbeta"]], [golden["loss"], golden["dloss_dbeta"]])
    assert np.count_nonzero(golden["z"]) > 0
