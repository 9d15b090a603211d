"""Convergence-driven mode on the GPU (csc_code_tol, csc_learn_tol and the
tau rule of the alternation) against the oracle's stopping rules.

The stopping decisions are compared exactly, so the tolerances are placed
away from the decision boundaries: the ADMM tolerance at the geometric mean
of two consecutive values of the oracle's residual history where it drops by
more than 10%, the CG tolerance at a value whose oracle step counts do not
change under a +-1% perturbation (checked in the test), and tau against
relative objective changes at least 5% away from it.  The one exception is
the first, cold CG solve of a learning call (about 40 steps), where float32
may need up to 3 more steps.  Iterates are held to the fixed-count
tolerances (codes 1e-4, filters 1e-4)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CODE_TOL = 1e-4


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_code_until_stops_with_the_oracle(lib):
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg, n=2)
    K, npix = cfg.k, b.shape[2] * b.shape[3]
    full = oracle.code(b, d, cfg.beta, cfg.rho, 30)
    worst = np.maximum(full["resid"][:, :, 0] / np.sqrt(K * npix),
                       full["resid"][:, :, 1] / np.sqrt(npix)).max(axis=1)
    k = int(np.argmax(worst[1:] < 0.9 * worst[:-1])) + 1      # first drop by more than 10%
    assert worst[k] < 0.9 * worst[k - 1] and np.all(worst[:k] > worst[k])
    tol = float(np.sqrt(worst[k] * worst[k - 1]))
    ref = oracle.code(b, d, cfg.beta, cfg.rho, 30, tol=tol)
    assert ref["iters"] == k + 1
    z, th, resid, _, done = lib.code_until(T(b), T(d), cfg.beta, cfg.rho, 30, tol, want_theta=True,
                                           want_resid=True)
    assert done == ref["iters"]
    assert np.abs(N(z) - ref["z"]).max() <= CODE_TOL
    assert np.abs(N(th) - ref["theta"]).max() <= CODE_TOL
    np.testing.assert_allclose(N(resid)[:, :, :2], ref["resid"], rtol=1e-3, atol=1e-5)
    # a tolerance that never fires runs the full count, like csc_code
    z2, _, _, _, done2 = lib.code_until(T(b), T(d), cfg.beta, cfg.rho, 6, 1e-30)
    assert done2 == 6
    z6 = lib.code(T(b), T(d), cfg.beta, cfg.rho, 6)[0]
    assert np.array_equal(N(z2), N(z6))


def _apply_learning_operator(g, z, mu, fsupp):
    """(I + sum_k 1/(2 mu_k) Z_k S^T S Z_k^T) g for one channel, from the
    oracle's correlation and reconstruction (eq:Learning_gamma)."""
    u = sum(oracle.csc._corr_crop(g[n], z[n], fsupp, 2) for n in range(g.shape[0]))   # S Z_k^T g: [K][1][*fs]
    return g + oracle.reconstruct(u / (2.0 * np.asarray(mu)).reshape(-1, 1, 1, 1), z)


def test_learn_until_cold_solve_is_valid(lib):
    """One multiplier update with cg_tol = 0.02 from gamma = 0 (about 40 CG
    steps).  A stopped solve is one of many valid ones, so instead of equal
    iterates: the GPU's step count is within 3 of the oracle's (float32's
    recursive residual drifts over that many steps), its gamma meets the rule
    on the oracle's operator (true residual within 1.2 tol: the recursive
    residual the decision reads is float32), and its filters and multipliers
    are the oracle's functions of that gamma.  The filters are badly
    conditioned in gamma near the solution (S Z^T gamma is small next to its
    terms), and the returned gamma passes a float32 inverse FFT (~7e-7
    relative over 12 stages) after the filters were formed from its
    spectrum, so they are held to twice the oracle's own filter change under
    a 1e-6 relative perturbation of gamma."""
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg, n=2)
    z = oracle.code(b, d0, cfg.beta, cfg.rho, 10)["z"].astype(np.float32)
    tol = 2e-2
    info = {}
    oracle.learn(b, z, cfg.fsupp, np.ones(cfg.k), None, 1, 80, cg_tol=tol, info=info)
    d, mu, gamma, got = lib.learn_until(T(b), T(z), cfg.fsupp, None, None, 1, 80, tol)
    assert abs(got[0] - info["cg_counts"][0]) <= 3, (got, info)
    g = N(gamma)
    res = -b.astype(np.float64) - _apply_learning_operator(g, z.astype(np.float64), np.ones(cfg.k), cfg.fsupp)
    assert np.linalg.norm(res) <= 1.2 * tol * np.linalg.norm(b), np.linalg.norm(res) / np.linalg.norm(b)
    d_ref, mu_ref, _ = oracle.learn(b, z, cfg.fsupp, np.ones(cfg.k), g, 1, 0)
    rng = np.random.default_rng(5)
    d_pert, _, _ = oracle.learn(b, z, cfg.fsupp, np.ones(cfg.k), g * (1 + 1e-6 * rng.standard_normal(g.shape)), 1, 0)
    bound = 2.0 * np.abs(d_pert - d_ref).max()
    assert bound < 0.05 * np.abs(d_ref).max()              # the bound still says something
    assert np.abs(N(d) - d_ref).max() <= bound, (np.abs(N(d) - d_ref).max(), bound)
    np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-3)


def test_learn_until_warm_counts_match_the_oracle(lib):
    """cg_tol = 0.02 over four multiplier updates: the warm-started solves
    stop after the oracle's 6-8 steps exactly (the counts do not change under
    a +-1% change of the tolerance); the cold first solve is within 3."""
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg, n=2)
    z = oracle.code(b, d0, cfg.beta, cfg.rho, 10)["z"].astype(np.float32)
    tol = 2e-2
    counts = []
    for f in (0.99, 1.0, 1.01):
        info = {}
        oracle.learn(b, z, cfg.fsupp, np.ones(cfg.k), None, 4, 60, cg_tol=tol * f, info=info)
        counts.append(info["cg_counts"])
    assert counts[0] == counts[1] == counts[2], counts     # no decision near the boundary
    ref = counts[1]
    _, _, _, got = lib.learn_until(T(b), T(z), cfg.fsupp, None, None, 4, 60, tol)
    assert got[1:] == ref[1:], (got, ref)
    assert abs(got[0] - ref[0]) <= 3, (got, ref)
    assert max(got[1:]) <= 10 < got[0]                     # warm starts take a few steps


def test_alternation_tau_stops_with_the_oracle(lib):
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg, n=2)
    tau = 0.05
    ref = oracle.learn_dictionary(b, d0, cfg.beta, cfg.rho, 5, 12, 3, 5, tau=tau)
    f = np.array(ref["objectives"][1::2])
    rel = np.abs(np.diff(f)) / np.abs(f[:-1])
    assert np.all(np.abs(rel - tau) > 0.05 * tau)            # every decision has a margin
    out = lib.learn_dictionary(T(b), T(d0), cfg.beta, cfg.rho, 5, 12, 3, 5, tau=tau)
    assert out["steps"] == ref["steps"] < 12
    assert np.abs(N(out["d"]) - ref["d"]).max() <= 1e-3


def _rand_case(seed, n, j, k, grid, fsupp, amp=10.0):
    rng = np.random.default_rng(seed)
    b = np.zeros((n, j) + grid, np.float32)
    for i in range(n):
        for c in range(j):
            b[i, c] = synth.contrast_normalize(synth.one_over_f(rng, grid)) * amp
    return b, synth.unit_filters(k, j, fsupp, seed + 1)


@pytest.mark.parametrize("grid,fsupp", [((64, 64), (11, 11)), ((8, 16, 16), (3, 5, 5))])
def test_code_until_colour_and_3d(lib, grid, fsupp):
    """The ADMM stopping rule with J = 3 on a 2-D grid and on a 3-D grid (the
    colour image and video forms): the GPU stops at the oracle's iteration
    (tolerance placed between two residual values that differ by more than
    10%), with the oracle's codes."""
    b, d = _rand_case(61, 2, 3, 5, grid, fsupp)
    K, npix, J = 5, int(np.prod(grid)), 3
    full = oracle.code(b, d, 0.5, 10.0, 30)
    worst = np.maximum(full["resid"][:, :, 0] / np.sqrt(K * npix),
                       full["resid"][:, :, 1] / np.sqrt(J * npix)).max(axis=1)
    k = int(np.argmax(worst[1:] < 0.9 * worst[:-1])) + 1
    assert worst[k] < 0.9 * worst[k - 1] and np.all(worst[:k] > worst[k])
    tol = float(np.sqrt(worst[k] * worst[k - 1]))
    ref = oracle.code(b, d, 0.5, 10.0, 30, tol=tol)
    assert ref["iters"] == k + 1
    z, _, _, _, done = lib.code_until(T(b), T(d), 0.5, 10.0, 30, tol)
    assert done == ref["iters"]
    assert np.abs(N(z) - ref["z"]).max() <= CODE_TOL


def test_learn_until_3d_colour(lib):
    """CG stopping rule on the 3-D, J = 3 form: a tolerance that never fires
    runs csc_learn's iteration (equal filters, bit for bit), and a firing one
    stops its cold solve within 3 steps of the oracle's count."""
    fs = (3, 5, 5)
    b, d0 = _rand_case(71, 2, 3, 4, (8, 16, 16), fs)
    z = oracle.code(b, d0, 0.5, 10.0, 10)["z"].astype(np.float32)
    d_fix, _, _ = lib.learn(T(b), T(z), fs, None, None, 2, 6)
    d_tol, _, _, counts = lib.learn_until(T(b), T(z), fs, None, None, 2, 6, 1e-30)
    assert counts == [6, 6]
    assert np.array_equal(N(d_tol), N(d_fix))
    info = {}
    oracle.learn(b, z, fs, np.ones(4), None, 1, 80, cg_tol=2e-2, info=info)
    _, _, _, got = lib.learn_until(T(b), T(z), fs, None, None, 1, 80, 2e-2)
    assert abs(got[0] - info["cg_counts"][0]) <= 3, (got, info)
