"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical float32 inputs.

Tolerances (tests/tolerances.py): codes within 1e-4 max-abs of the oracle
after a fixed iteration count, objectives within 1e-5 relative.  Inputs whose
codes exceed |z| ~ 30 use 3e-6 * max|z| instead, and the chained alternation
uses bounds tied to a measured float32 floor (tests/test_float32_floor.py).
Every coding comparison also asserts a non-zero code density so that an
all-zero result cannot pass.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tolerances import (CHAIN_CODE_TOL, CHAIN_FILTER_TOL, CHAIN_MU_RTOL, CHAIN_OBJ_RTOL, CODE_TOL, OBJ_RTOL,
                        code_tol)

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def density(z):
    return np.count_nonzero(z) / z.size


def rand_case(seed, n, j, k, grid, fsupp, amp=10.0):
    rng = np.random.default_rng(seed)
    b = np.zeros((n, j) + grid, np.float32)
    for i in range(n):
        for c in range(j):
            f = synth.contrast_normalize(synth.one_over_f(rng, grid[-2:] if len(grid) == 2 else grid)) * amp
            b[i, c] = f
    d = synth.unit_filters(k, j, fsupp, seed + 1)
    return b, d


# ----------------------------------------------------------------- coding

@pytest.mark.parametrize("name", ["small", "small_rho01"])
def test_code_small_config(lib, name):
    cfg = synth.CONFIGS[name]
    b, d = synth.make_inputs(cfg)
    ref = oracle.code(b, d, cfg.beta, cfg.rho, cfg.t_in)
    z, _, _, _ = lib.code(T(b), T(d), cfg.beta, cfg.rho, cfg.t_in)
    zg = N(z)
    assert density(ref["z"]) > 0.01
    err = np.abs(zg - ref["z"]).max()
    assert err <= CODE_TOL, err


@pytest.mark.parametrize("grid,k,j,n", [
    ((64, 64), 5, 1, 3),        # odd K (one half-empty pair)
    ((32, 64), 6, 1, 2),        # rectangular tile
    ((16, 16), 3, 1, 2),        # smallest tile
    ((8, 32), 4, 1, 2),         # side 8: global path
    ((256, 256), 4, 1, 1),      # split path (row / column / row phases)
    ((128, 256), 3, 1, 1),      # split path, rectangular
    ((256, 128), 5, 1, 2),      # split path, tall, odd K
    ((256, 256), 25, 1, 8),     # split path, two pairs per row-phase group, last group partial, odd K
    ((128, 256), 4, 2, 2),      # split path, J = 2
    ((256, 256), 5, 3, 1),      # split path, J = 3, odd K
    ((64, 64), 6, 3, 2),        # tensor CSC, J = 3 (tile path)
    ((64, 64), 4, 2, 2),        # J = 2
    ((8, 16, 16), 4, 3, 1),     # 3-D volume, J = 3 (global path)
])
def test_code_shapes(lib, grid, k, j, n):
    fs = (3, 5, 5) if len(grid) == 3 else (min(11, grid[0]), min(11, grid[1]))
    b, d = rand_case(11 + k + j, n, j, k, grid, fs)
    beta, rho, iters = 1.0, 5.0, 12
    ref = oracle.code(b, d, beta, rho, iters)
    z, _, _, _ = lib.code(T(b), T(d), beta, rho, iters)
    assert density(ref["z"]) > 0.005
    err = np.abs(N(z) - ref["z"]).max()
    assert err <= code_tol(ref["z"]), (err, code_tol(ref["z"]))


def test_code_split_warm_start_theta(lib):
    """Warm start (z and theta both enter through the forward-only phase)
    and theta output on a 256 x 256 grid."""
    b, d = rand_case(7, 2, 1, 6, (256, 256), (11, 11))
    beta, rho = 1.0, 5.0
    first = oracle.code(b, d, beta, rho, 4)
    z0, th0 = first["z"].astype(np.float32), first["theta"].astype(np.float32)
    ref = oracle.code(b, d, beta, rho, 5, z0=z0, theta0=th0)
    z, th, resid, _ = lib.code(T(b), T(d), beta, rho, 5, z=T(z0), theta=T(th0), want_resid=True)
    assert density(ref["z"]) > 0.005
    assert np.abs(N(z) - ref["z"]).max() <= code_tol(ref["z"])
    assert np.abs(N(th) - ref["theta"]).max() <= code_tol(ref["theta"])
    r = N(resid)
    np.testing.assert_allclose(r[:, :, 0], ref["resid"][:, :, 0], rtol=1e-3, atol=1e-5)
    np.testing.assert_allclose(r[:, :, 1], ref["resid"][:, :, 1], rtol=1e-3, atol=1e-5)


def test_code_warm_start_theta_and_residuals(lib):
    b, d = rand_case(5, 3, 1, 8, (64, 64), (11, 11))
    beta, rho = 1.0, 10.0
    first = oracle.code(b, d, beta, rho, 6)
    z0, th0 = first["z"], first["theta"]
    ref = oracle.code(b, d, beta, rho, 9, z0=z0, theta0=th0)
    z = T(z0)
    th = T(th0)
    z, th, resid, _ = lib.code(T(b), T(d), beta, rho, 9, z=z, theta=th, want_resid=True)
    assert np.abs(N(z) - ref["z"]).max() <= CODE_TOL
    assert np.abs(N(th) - ref["theta"]).max() <= CODE_TOL
    r = N(resid)
    np.testing.assert_allclose(r[:, :, 0], ref["resid"][:, :, 0], rtol=1e-3, atol=1e-5)
    np.testing.assert_allclose(r[:, :, 1], ref["resid"][:, :, 1], rtol=1e-3, atol=1e-5)
    assert np.all(r[:, :, 2] == rho)


def test_code_zero_iterations_and_zero_codes(lib):
    import torch
    b, d = rand_case(3, 2, 1, 4, (32, 32), (5, 5))
    z, th, _, _ = lib.code(T(b), T(d), 1.0, 10.0, 0, want_theta=True)
    assert torch.count_nonzero(z).item() == 0 and torch.count_nonzero(th).item() == 0
    # beta so large that every code stays zero
    z, _, _, _ = lib.code(T(b), T(d), 1e6, 10.0, 5)
    assert torch.count_nonzero(z).item() == 0


def test_code_adaptive_rho_replayed(lib):
    """Adaptive rho: the GPU returns its rho schedule; the oracle replays it.
    Decisions taken right at the threshold may differ between float32 and
    float64 (parity of the decisions themselves is not asserted)."""
    cfg = synth.CONFIGS["learn"]
    b, d = synth.make_inputs(cfg, n=3)
    z, _, resid, rho = lib.code(T(b), T(d), cfg.beta, cfg.rho0, cfg.t_in, adaptive=True, want_resid=True)
    r = N(resid)
    sched = np.concatenate([r[:, :, 2], N(rho)[None]], axis=0)
    assert (sched != cfg.rho0).any()
    ref = oracle.code(b, d, cfg.beta, cfg.rho0, cfg.t_in, rho_schedule=sched)
    assert density(ref["z"]) > 0.01
    err = np.abs(N(z) - ref["z"]).max()
    assert err <= CODE_TOL, err
    own = oracle.code(b, d, cfg.beta, cfg.rho0, cfg.t_in, adaptive=True)
    agree = (own["rho"] == sched).mean()
    assert agree > 0.9


# -------------------------------------------------------------- objective

@pytest.mark.parametrize("grid,j", [((64, 64), 1), ((128, 128), 1), ((256, 256), 1), ((64, 64), 3),
                                    ((8, 16, 16), 3)])
def test_objective(lib, grid, j):
    k = 6
    fs = (3, 5, 5) if len(grid) == 3 else (11, 11)
    b, d = rand_case(21, 2, j, k, grid, fs)
    z = oracle.code(b, d, 1.0, 5.0, 8)["z"].astype(np.float32)
    per, tot = oracle.objective(b, d, z, 0.7)
    out = N(lib.objective(T(b), T(d), T(z), 0.7))
    np.testing.assert_allclose(out[:-1], per, rtol=OBJ_RTOL)
    assert abs(out[-1] - tot) <= OBJ_RTOL * abs(tot)


# --------------------------------------------------------------- learning

def learn_tol(d_ref):
    return 1e-4 * max(1.0, float(np.abs(d_ref).max()))


@pytest.mark.parametrize("form", ["span", "direct"])
@pytest.mark.parametrize("grid,j,k", [((64, 64), 1, 8), ((64, 64), 1, 7), ((64, 64), 2, 6), ((32, 64), 3, 6),
                                      ((128, 128), 3, 5), ((256, 256), 1, 4)])
def test_learn(lib, grid, j, k, form):
    """Both forms of the learning CG against the oracle."""
    b, d0 = rand_case(31 + k, 3, j, k, grid, (11, 11))
    z = oracle.code(b, d0, 1.0, 5.0, 10)["z"].astype(np.float32)
    assert density(z) > 0.005
    mu0 = np.linspace(0.8, 1.5, k)
    d_ref, mu_ref, g_ref = oracle.learn(b, z, (11, 11), mu0.astype(np.float32), None, 3, 6)
    d, mu, gamma = lib.learn(T(b), T(z), (11, 11), T(mu0), None, 3, 6, form=form)
    assert np.abs(N(d) - d_ref).max() <= learn_tol(d_ref)
    np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
    assert np.abs(N(gamma) - g_ref).max() <= 1e-4 * max(1.0, np.abs(g_ref).max())


def test_learn_3d(lib):
    """Learning on a 3-D grid with J = 3 (the colour video form): the general
    path (axis FFTs, support crop of a 3-D tile)."""
    fs = (3, 5, 5)
    b, d0 = rand_case(51, 2, 3, 4, (8, 16, 16), fs)
    z = oracle.code(b, d0, 1.0, 5.0, 10)["z"].astype(np.float32)
    assert density(z) > 0.005
    mu0 = np.linspace(0.8, 1.5, 4)
    d_ref, mu_ref, g_ref = oracle.learn(b, z, fs, mu0.astype(np.float32), None, 3, 6)
    d, mu, gamma = lib.learn(T(b), T(z), fs, T(mu0), None, 3, 6)
    assert np.abs(N(d) - d_ref).max() <= learn_tol(d_ref)
    np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
    assert np.abs(N(gamma) - g_ref).max() <= 1e-4 * max(1.0, np.abs(g_ref).max())


def test_learn_warm_gamma(lib):
    b, d0 = rand_case(41, 2, 1, 6, (64, 64), (11, 11))
    z = oracle.code(b, d0, 1.0, 5.0, 10)["z"].astype(np.float32)
    _, mu1, g1 = oracle.learn(b, z, (11, 11), np.ones(6), None, 2, 5)
    g1 = g1.astype(np.float32)
    mu1 = mu1.astype(np.float32)
    d_ref, mu_ref, g_ref = oracle.learn(b, z, (11, 11), mu1, g1, 2, 5)
    for form in ("span", "direct"):
        d, mu, gamma = lib.learn(T(b), T(z), (11, 11), T(mu1), T(g1), 2, 5, form=form)
        assert np.abs(N(d) - d_ref).max() <= learn_tol(d_ref)
        np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
        assert np.abs(N(gamma) - g_ref).max() <= 1e-4 * max(1.0, np.abs(g_ref).max())


@pytest.mark.parametrize("inner,cg", [(2, 0), (1, 1), (1, 3)])
def test_learn_short_counts(lib, inner, cg):
    """Edge counts of the learning loop in both forms: no CG step (the
    filters follow from the warm start alone), a single step, a single
    multiplier update."""
    b, d0 = rand_case(61, 2, 1, 5, (64, 64), (11, 11))
    z = oracle.code(b, d0, 1.0, 5.0, 10)["z"].astype(np.float32)
    _, mu1, g1 = oracle.learn(b, z, (11, 11), np.ones(5), None, 1, 4)
    g1 = g1.astype(np.float32)
    mu1 = mu1.astype(np.float32)
    d_ref, mu_ref, g_ref = oracle.learn(b, z, (11, 11), mu1, g1, inner, cg)
    for form in ("span", "direct"):
        d, mu, gamma = lib.learn(T(b), T(z), (11, 11), T(mu1), T(g1), inner, cg, form=form)
        assert np.abs(N(d) - d_ref).max() <= learn_tol(d_ref), form
        np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
        assert np.abs(N(gamma) - g_ref).max() <= 1e-4 * max(1.0, np.abs(g_ref).max()), form


# ------------------------------------------------------------ alternation

def test_learn_dictionary_small_config(lib):
    """Alg. 1 on the 4 x 64x64, K=16 workload: 2 outer steps of 20 coding
    iterations and learning (10 mu steps x 10 CG steps).

    Each half step is compared with the oracle started from the GPU's own
    state (identical float32 inputs): codes within 1e-4, filters within 1e-4.
    The chained run (each side feeding itself) is compared with the oracle's
    chained run at the bounds tied to the float32 floor of this workload
    (tests/tolerances.py): codes, filters and multipliers at the end, the
    objective after every half step."""
    import torch
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg)
    bt = T(b)
    d = T(d0)
    z = theta = gamma = None
    mu = torch.ones(cfg.k, dtype=torch.float32, device="cuda")
    for step in range(cfg.t_out):
        z_in = None if z is None else N(z).astype(np.float32)
        th_in = None if theta is None else N(theta).astype(np.float32)
        d_in = N(d).astype(np.float32)
        ref = oracle.code(b, d_in, cfg.beta, cfg.rho, cfg.t_in, z0=z_in, theta0=th_in)
        z, theta, _, _ = lib.code(bt, d, cfg.beta, cfg.rho, cfg.t_in, z=z, theta=theta, want_theta=True)
        assert density(ref["z"]) > 0.01
        ez = np.abs(N(z) - ref["z"]).max()
        zf = N(z).astype(np.float32)
        mu_in = N(mu).astype(np.float32)
        g_in = None if gamma is None else N(gamma).astype(np.float32)
        d_ref, mu_ref, _ = oracle.learn(b, zf, cfg.fsupp, mu_in, g_in, cfg.learn_inner, cfg.learn_cg)
        d, mu, gamma = lib.learn(bt, z, cfg.fsupp, mu, gamma, cfg.learn_inner, cfg.learn_cg)
        ed = np.abs(N(d) - d_ref).max()
        emu = np.abs(N(mu) / mu_ref - 1).max()
        print("half steps of outer step %d from the GPU's state: codes %.2e, filters %.2e, mu %.2e"
              % (step, ez, ed, emu))
        assert ez <= CODE_TOL, step
        assert ed <= 1e-4, step
        assert emu <= 1e-4, step

    ref = oracle.learn_dictionary(b, d0, cfg.beta, cfg.rho, cfg.t_in, cfg.t_out, cfg.learn_inner, cfg.learn_cg)
    out = lib.learn_dictionary(bt, T(d0), cfg.beta, cfg.rho, cfg.t_in, cfg.t_out, cfg.learn_inner, cfg.learn_cg)
    ez = np.abs(N(out["z"]) - ref["z"]).max()
    ed = np.abs(N(out["d"]) - ref["d"]).max()
    emu = np.abs(N(out["mu"]) / ref["mu"] - 1).max()
    eobj = np.abs(N(out["objectives"]) / np.asarray(ref["objectives"]) - 1)
    print("chained run: codes %.2e (bound %.1e), filters %.2e (%.1e), mu %.2e (%.1e), objective per half step %s (%.1e)"
          % (ez, CHAIN_CODE_TOL, ed, CHAIN_FILTER_TOL, emu, CHAIN_MU_RTOL,
             " ".join("%.2e" % e for e in eobj), CHAIN_OBJ_RTOL))
    assert density(ref["z"]) > 0.01
    assert ez <= CHAIN_CODE_TOL
    assert ed <= CHAIN_FILTER_TOL
    assert emu <= CHAIN_MU_RTOL
    assert eobj.max() <= CHAIN_OBJ_RTOL
    # the GPU's objective of its own final state against the oracle's objective of that state
    _, f_own = oracle.objective(b, N(out["d"]), N(out["z"]), cfg.beta)
    assert abs(N(out["objectives"])[-1] - f_own) <= OBJ_RTOL * f_own
