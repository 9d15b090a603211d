"""Parity at the extremes of the scaling sweeps (bench.py --sweep; the
shapes of the paper's scalability study, Sec. 4.4, and its tensor study,
Sec. 4.5) and one full-size outer step of tensor CSC.

Learning is joint over images, so the learning checks run the whole
workload: the GPU's learning from the GPU's codes against the oracle's
learning from the same (float32) codes, with fewer multiplier updates and CG
steps than the benchmark (the oracle's cost grows with N K per step).
Tolerances as the other parity tests: filters 1e-4 of max(1, max|d|), mu
1e-4 relative, codes 1e-4 (or 3e-6 max|z|), objective 1e-5 relative."""
import numpy as np
import pytest

import oracle
import synth
from tolerances import OBJ_RTOL, code_tol

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def sweep_point(name, **match):
    for cfg in synth.SWEEPS[name]:
        if all(getattr(cfg, k) == v for k, v in match.items()):
            return cfg
    raise KeyError(name)


def check_learning(lib, b, z, fsupp, k, inner, cg):
    d, mu, _ = lib.learn(T(b), z, fsupp, None, None, inner, cg)
    zf = N(z).astype(np.float32)
    d_ref, mu_ref, _ = oracle.learn(b, zf, fsupp, np.ones(k), None, inner, cg)
    err = np.abs(N(d) - d_ref).max() / max(1.0, np.abs(d_ref).max())
    print("learning: filters %.2e, mu %.2e" % (err, np.abs(N(mu) / mu_ref - 1).max()), flush=True)
    assert err <= 1e-4, err
    np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
    return d


def test_gray_sweep_100_images(lib):
    """gray_N at N = 100 (128^2, K = 100): 10 coding iterations with adaptive
    rho from 10 (the sweep's setting), two sampled images against the oracle
    replaying the GPU's rho schedule, then learning 2 x 4 from the codes of
    all 100 images."""
    cfg = sweep_point("gray_N", n=100)
    b, d0 = synth.make_inputs(cfg)
    print("gray_N N=100", flush=True)
    z, _, resid, rho = lib.code(T(b), T(d0), cfg.beta, cfg.rho0, cfg.t_in, adaptive=True, want_resid=True)
    zn = N(z)
    sched = np.concatenate([N(resid)[:, :, 2], N(rho)[None]], axis=0)
    for i in (0, cfg.n - 1):
        ref = oracle.code(b[i:i + 1], d0, cfg.beta, cfg.rho0, cfg.t_in, rho_schedule=sched[:, i:i + 1])["z"]
        assert np.count_nonzero(ref) / ref.size > 0.005
        assert np.abs(zn[i:i + 1] - ref).max() <= code_tol(ref), i
    check_learning(lib, b, z, cfg.fsupp, cfg.k, 2, 4)


def test_rgb_sweep_100_filters(lib):
    """rgb_K at K = 100 (10 RGB images 128^2, filters 11x11x3): 20 coding
    iterations (two sampled images against the oracle), learning 2 x 5."""
    cfg = sweep_point("rgb_K", k=100)
    b, d0 = synth.make_inputs(cfg)
    print("rgb_K K=100", flush=True)
    z, _, _, _ = lib.code(T(b), T(d0), cfg.beta, cfg.rho, cfg.t_in)
    zn = N(z)
    for i in (0, cfg.n - 1):
        ref = oracle.code(b[i:i + 1], d0, cfg.beta, cfg.rho, cfg.t_in)["z"]
        assert np.count_nonzero(ref) / ref.size > 0.005
        assert np.abs(zn[i:i + 1] - ref).max() <= code_tol(ref), i
    check_learning(lib, b, z, cfg.fsupp, cfg.k, 2, 5)


def test_tensor_full_size_outer_step(lib):
    """One outer step of Alg. 1 on the full tensor workload (32 RGB images
    128^2, K = 64 filters 11x11x3, beta 0.5, rho 10): coding 20 iterations
    from zero, learning (3 x 5 here) from those codes, and the objective of
    the learned filters with those codes, each against the oracle."""
    cfg = synth.CONFIGS["tensor"]
    b, d0 = synth.make_inputs(cfg)
    print("tensor outer step", flush=True)
    z, _, _, _ = lib.code(T(b), T(d0), cfg.beta, cfg.rho, cfg.t_in)
    zn = N(z)
    ref = oracle.code(b[5:6], d0, cfg.beta, cfg.rho, cfg.t_in)["z"]
    assert np.abs(zn[5:6] - ref).max() <= code_tol(ref)
    d = check_learning(lib, b, z, cfg.fsupp, cfg.k, 3, 5)
    obj = N(lib.objective(T(b), d, z, cfg.beta))
    per, tot = oracle.objective(b, N(d).astype(np.float32), zn.astype(np.float32), cfg.beta)
    np.testing.assert_allclose(obj[:-1], per, rtol=OBJ_RTOL)
    assert abs(obj[-1] - tot) <= OBJ_RTOL * abs(tot)
