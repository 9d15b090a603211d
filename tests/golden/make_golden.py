"""Writes oracle_tiny.json: the FP64 oracle's results on one tiny, fully
stored problem (coding, learning, objective, unrolled-loss gradients).

The file pins the oracle to its own earlier output: a later change to the
oracle's arithmetic shows up in tests/test_golden.py and must be justified
against the paper before this file is rewritten.  Only oracle/ is called
(the inputs are drawn here with numpy and stored in the file).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def inputs():
    """One 16 x 16 image of i.i.d. normal values times 10 and two 3 x 3
    unit-norm filters, rounded to float32."""
    rng = np.random.default_rng(20170927)
    b = (10.0 * rng.standard_normal((1, 1, 16, 16))).astype(np.float32)
    d = rng.standard_normal((2, 1, 3, 3))
    d /= np.sqrt((d ** 2).sum(axis=(1, 2, 3), keepdims=True))
    return b, d.astype(np.float32)


def compute(b, d):
    beta, rho = 2.0, 2.0
    c = oracle.code(b, d, beta, rho, 6)
    dl, mu, gamma = oracle.learn(b, c["z"].astype(np.float32), (3, 3), np.ones(2), None, 2, 3)
    per, tot = oracle.objective(b, d, c["z"].astype(np.float32), beta)
    L, gd, gb = oracle.code_loss_grad(b, d, beta, rho, 6)
    return {
        "beta": beta, "rho": rho, "code_iters": 6, "learn_inner": 2, "learn_cg": 3,
        "z": c["z"].ravel().tolist(), "theta": c["theta"].ravel().tolist(),
        "resid": c["resid"].ravel().tolist(),
        "d_learned": dl.ravel().tolist(), "mu": np.asarray(mu).ravel().tolist(),
        "gamma": gamma.ravel().tolist(),
        "objective": [float(x) for x in per] + [float(tot)],
        "loss": float(L), "dloss_dd": gd.ravel().tolist(), "dloss_dbeta": float(gb),
    }


if __name__ == "__main__":
    b, d = inputs()
    out = {"b": b.ravel().tolist(), "b_shape": list(b.shape), "d": d.ravel().tolist(), "d_shape": list(d.shape)}
    out.update(compute(b, d))
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as f:
        json.dump(out, f)
    print("wrote", os.path.join(HERE, "oracle_tiny.json"))
