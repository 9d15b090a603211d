"""Pins for the FP64 oracle: each check compares it with something other than
itself -- dense matrices built tap by tap, brute-force spatial sums, closed
forms and invariants the paper's equations imply.

Dense helpers here are written independently of ``oracle`` (explicit loops,
no FFT), so a dropped term, a wrong sign, a conjugation or a transposed
operand in the oracle makes one of these fail.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- dense tools

def conv_matrix(dk, grid):
    """Dense D x D matrix of circular convolution with filter dk (corner
    anchored): (D_k z)[p] = sum_m dk[m] z[(p - m) mod grid]."""
    D = int(np.prod(grid))
    A = np.zeros((D, D))
    pts = list(itertools.product(*[range(g) for g in grid]))
    idx = {p: i for i, p in enumerate(pts)}
    for p in pts:
        for m in itertools.product(*[range(s) for s in dk.shape]):
            q = tuple((pi - mi) % g for pi, mi, g in zip(p, m, grid))
            A[idx[p], idx[q]] += dk[m]
    return A


def dict_matrix(d, grid):
    """Block matrix D of size JD x KD (Sec. 3.3): block (j, k) = conv(d[k, j])."""
    K, J = d.shape[:2]
    rows = []
    for j in range(J):
        rows.append(np.hstack([conv_matrix(d[k, j], grid) for k in range(K)]))
    return np.vstack(rows)


def brute_conv(d, z):
    """Spatial brute-force sum_k d_jk * z_k for one image: z [K][*grid]."""
    K, J = d.shape[:2]
    grid = z.shape[1:]
    out = np.zeros((J,) + grid)
    for j in range(J):
        for k in range(K):
            for m in itertools.product(*[range(s) for s in d.shape[2:]]):
                out[j] += d[k, j][m] * np.roll(z[k], shift=m, axis=tuple(range(len(grid))))
    return out


def dense_admm(x, Dm, beta, rho, iters, z=None, th=None):
    """eq:Inference_solution with explicit matrices (one image, x of length JD)."""
    KD = Dm.shape[1]
    z = np.zeros(KD) if z is None else z.copy()
    th = np.zeros(KD) if th is None else th.copy()
    A = Dm @ Dm.T + np.eye(Dm.shape[0]) / rho
    hist = []
    for _ in range(iters):
        lam = np.linalg.solve(A, Dm @ th + Dm @ z / rho - x / rho)
        v = Dm.T @ lam
        th_new = np.clip(v - z / rho, -beta, beta)
        z_new = z + rho * (th_new - v)
        hist.append(dict(lam=lam, r_pri=np.linalg.norm(th_new - v),
                         r_dual=rho * np.linalg.norm(Dm @ (th_new - th)),
                         z=z_new, th=th_new, z_prev=z, th_prev=th))
        z, th = z_new, th_new
    return z, th, hist


def rand_filters(K, J, fs, rng=RNG):
    d = rng.standard_normal((K, J) + fs)
    return d / np.sqrt((d.reshape(K, -1) ** 2).sum(1)).reshape((K,) + (1,) * (d.ndim - 1))


# ------------------------------------------------------------------ P1 / P13

@pytest.mark.parametrize("grid,fs,J", [((8, 8), (3, 3), 1), ((16, 12), (5, 4), 1),
                                        ((6, 8, 8), (2, 3, 3), 1), ((8, 8), (3, 3), 3)])
def test_convolution_convention_bruteforce(grid, fs, J):
    K = 3
    d = rand_filters(K, J, fs)
    z = RNG.standard_normal((2, K) + grid)
    rec = oracle.reconstruct(d, z)
    for n in range(2):
        np.testing.assert_allclose(rec[n], brute_conv(d, z[n]), atol=1e-12, rtol=0)


def test_objective_bruteforce():
    grid, fs, K, J = (8, 10), (3, 3), 3, 2
    d = rand_filters(K, J, fs)
    z = RNG.standard_normal((2, K) + grid) * (RNG.random((2, K) + grid) < 0.3)
    b = RNG.standard_normal((2, J) + grid)
    beta = 0.7
    per, tot = oracle.objective(b, d, z, beta)
    for n in range(2):
        res = b[n] - brute_conv(d, z[n])
        ref = 0.5 * (res ** 2).sum() + beta * np.abs(z[n]).sum()
        assert abs(per[n] - ref) <= 1e-12 * abs(ref)
    assert abs(tot - per.sum()) <= 1e-12 * abs(tot)


def test_parseval_scaling():
    x = RNG.standard_normal((16, 8))
    xh = np.fft.fftn(x)
    assert abs((x ** 2).sum() - (np.abs(xh) ** 2).sum() / x.size) < 1e-12 * (x ** 2).sum()


# ------------------------------------------------------------- P3 / P6 coding

@pytest.mark.parametrize("J", [1, 2, 3])
def test_coding_matches_dense_admm(J):
    grid, fs, K = (6, 6), (3, 3), 2
    d = rand_filters(K, J, fs)
    b = RNG.standard_normal((1, J) + grid) * 2
    beta, rho, T = 0.3, 1.7, 12
    Dm = dict_matrix(d, grid)
    z_ref, th_ref, hist = dense_admm(b[0].reshape(-1), Dm, beta, rho, T)
    out = oracle.code(b, d, beta, rho, T)
    np.testing.assert_allclose(out["z"][0].reshape(-1), z_ref, atol=1e-12)
    np.testing.assert_allclose(out["theta"][0].reshape(-1), th_ref, atol=1e-12)
    res_ref = np.array([[h["r_pri"], h["r_dual"]] for h in hist])
    np.testing.assert_allclose(out["resid"][:, 0], res_ref, rtol=1e-10, atol=1e-13)
    assert np.count_nonzero(out["z"]) > 0


def test_coding_warm_start_matches_dense():
    grid, fs, K, J = (6, 6), (3, 3), 3, 1
    d = rand_filters(K, J, fs)
    b = RNG.standard_normal((2, J) + grid) * 3
    z0 = RNG.standard_normal((2, K) + grid) * (RNG.random((2, K) + grid) < 0.3)
    th0 = np.clip(RNG.standard_normal((2, K) + grid), -0.4, 0.4)
    beta, rho, T = 0.4, 0.9, 7
    out = oracle.code(b, d, beta, rho, T, z0=z0, theta0=th0)
    Dm = dict_matrix(d, grid)
    for n in range(2):
        z_ref, th_ref, _ = dense_admm(b[n].reshape(-1), Dm, beta, rho, T,
                                      z0[n].reshape(-1), th0[n].reshape(-1))
        np.testing.assert_allclose(out["z"][n].reshape(-1), z_ref, atol=1e-12)
        np.testing.assert_allclose(out["theta"][n].reshape(-1), th_ref, atol=1e-12)


def test_residual_identity_and_dual_sign():
    """rho D (theta^i - theta^{i+1}) = lam^{i+1} + x - D z^{i+1}; at the fixed
    point lam* = D z* - x (the dual optimum of eq:Inference_Dual)."""
    grid, fs, K = (6, 6), (3, 3), 2
    d = rand_filters(K, 1, fs)
    x = RNG.standard_normal(36) * 2
    Dm = dict_matrix(d, grid)
    rho = 1.3
    _, _, hist = dense_admm(x, Dm, 0.2, rho, 5000)
    for h in hist[:20]:
        lhs = rho * Dm @ (h["th_prev"] - h["th"])
        rhs = h["lam"] + x - Dm @ h["z"]
        np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    h = hist[-1]
    np.testing.assert_allclose(h["lam"], Dm @ h["z"] - x, atol=1e-8)
    # and the oracle reaches the same point
    out = oracle.code(x.reshape(1, 1, *grid), d, 0.2, rho, 5000)
    np.testing.assert_allclose(out["z"][0].reshape(-1), h["z"], atol=1e-10)


def test_moreau_soft_threshold_form():
    """z + rho (clip(v - z/rho, +-beta) - v) == soft(z - rho v, rho beta)."""
    z = RNG.standard_normal(1000) * 3
    v = RNG.standard_normal(1000) * 2
    rho, beta = 2.5, 0.6
    lhs = z + rho * (np.clip(v - z / rho, -beta, beta) - v)
    np.testing.assert_allclose(lhs, oracle.soft(z - rho * v, rho * beta), atol=1e-12)
    # soft threshold closed form on a few points
    assert oracle.soft(np.array([3.0, -3.0, 0.5, -0.5]), 1.0).tolist() == [2.0, -2.0, 0.0, -0.0]


@pytest.mark.parametrize("J", [1, 3])
def test_implicit_theta_form_equals_literal(J):
    grid, fs, K = (12, 12), (5, 5), 4
    d = rand_filters(K, J, fs)
    b = RNG.standard_normal((2, J) + grid) * 3
    z0 = RNG.standard_normal((2, K) + grid) * (RNG.random((2, K) + grid) < 0.2)
    th0 = np.clip(RNG.standard_normal((2, K) + grid), -0.5, 0.5)
    lit = oracle.code(b, d, 0.5, 2.0, 30, z0=z0, theta0=th0)
    imp = oracle.code_implicit(b, d, 0.5, 2.0, 30, z0=z0, theta0=th0)
    np.testing.assert_allclose(imp["z"], lit["z"], atol=1e-11)
    np.testing.assert_allclose(imp["theta"], lit["theta"], atol=1e-11)


# ------------------------------------------------------- P7 / P8 convergence

def test_kkt_at_convergence_and_residuals_vanish():
    grid, fs, K = (16, 16), (5, 5), 4
    d = rand_filters(K, 1, fs)
    b = RNG.standard_normal((1, 1) + grid) * 3
    beta, rho = 1.0, 1.0
    out = oracle.code(b, d, beta, rho, 3000)
    z = out["z"][0]
    g = np.zeros_like(z)
    Dm = dict_matrix(d, grid)
    g = (Dm.T @ (b[0, 0].reshape(-1) - Dm @ z.reshape(-1))).reshape(z.shape)
    on = z != 0
    assert on.sum() > 0
    np.testing.assert_allclose(g[on], beta * np.sign(z[on]), atol=1e-8)
    assert np.abs(g[~on]).max() <= beta + 1e-8
    r = out["resid"][:, 0]
    assert r[-1, 0] < 1e-8 * max(1.0, r[0, 0]) and r[-1, 1] < 1e-8 * max(1.0, r[0, 1])


def test_delta_filter_gives_soft_threshold():
    """K = 1 with a corner delta filter makes D the identity, so the lasso
    solution is soft(x, beta)."""
    grid = (16, 16)
    d = np.zeros((1, 1, 3, 3))
    d[0, 0, 0, 0] = 1.0
    b = RNG.standard_normal((2, 1) + grid) * 2
    out = oracle.code(b, d, 0.8, 2.0, 200)
    np.testing.assert_allclose(out["z"][:, 0], oracle.soft(b[:, 0], 0.8), atol=1e-12)


# ---------------------------------------------------------------- P9 tensor

def test_tensor_equal_channels_reduce_to_plain():
    """J equal channels x_j = x with d_jk = d_k / sqrt(J) give the codes of
    plain CSC on sqrt(J) x (sum_j ||x - Dz/sqrt J||^2 = ||sqrt J x - D z||^2 + c)."""
    grid, fs, K, J = (12, 12), (5, 5), 3, 3
    d1 = rand_filters(K, 1, fs)
    x = RNG.standard_normal((2, 1) + grid) * 3
    dJ = np.repeat(d1, J, axis=1) / np.sqrt(J)
    bJ = np.repeat(x, J, axis=1)
    a = oracle.code(bJ, dJ, 0.5, 1.5, 25)
    p = oracle.code(np.sqrt(J) * x, d1, 0.5, 1.5, 25)
    np.testing.assert_allclose(a["z"], p["z"], atol=1e-11)
    assert np.count_nonzero(p["z"]) > 0


def test_tensor_3d_matches_dense():
    grid, fs, K, J = (4, 4, 4), (2, 2, 2), 2, 2
    d = rand_filters(K, J, fs)
    b = RNG.standard_normal((1, J) + grid) * 2
    Dm = dict_matrix(d, grid)
    z_ref, th_ref, _ = dense_admm(b[0].reshape(-1), Dm, 0.3, 1.1, 6)
    out = oracle.code(b, d, 0.3, 1.1, 6)
    np.testing.assert_allclose(out["z"][0].reshape(-1), z_ref, atol=1e-12)


# ------------------------------------------------------------- adaptive rho

def test_adaptive_rho_replay_and_rule():
    grid, fs, K = (16, 16), (5, 5), 4
    d = rand_filters(K, 1, fs)
    b = RNG.standard_normal((3, 1) + grid) * 4
    out = oracle.code(b, d, 1.0, 10.0, 25, adaptive=True)
    sched, res = out["rho"], out["resid"]
    ratio = sched[1:] / sched[:-1]
    assert set(np.unique(np.round(ratio, 12))) <= {0.5, 1.0, 2.0}
    for i in range(25):
        for n in range(3):
            rp, rd = res[i, n]
            want = 2.0 if rp > 10 * rd else (0.5 if rd > 10 * rp else 1.0)
            assert ratio[i, n] == want
    assert (ratio != 1.0).any()
    rep = oracle.code(b, d, 1.0, 10.0, 25, rho_schedule=sched)
    np.testing.assert_array_equal(rep["z"], out["z"])


# -------------------------------------------------------- P10 / P11 learning

def learning_dense(x, z, fs, mu):
    """Primal ridge of eq:Learning_new by dense normal equations for one
    channel: argmin_d 1/2 ||x - Z S^T d||^2 + sum_k mu_k ||d_k||^2.
    x [N][*grid], z [N][K][*grid] -> d [K][*fs]."""
    N, K = z.shape[:2]
    grid = z.shape[2:]
    M = int(np.prod(fs))
    cols = []
    for k in range(K):
        for m in itertools.product(*[range(s) for s in fs]):
            col = np.concatenate([np.roll(z[n, k], shift=m, axis=tuple(range(len(grid)))).reshape(-1)
                                  for n in range(N)])
            cols.append(col)
    W = np.array(cols).T                                   # ND x KM
    reg = np.repeat(2 * np.asarray(mu), M)
    dvec = np.linalg.solve(W.T @ W + np.diag(reg), W.T @ x.reshape(-1))
    return dvec.reshape((K,) + tuple(fs)), W


def test_learning_dual_equals_primal_ridge():
    N, K, grid, fs = 2, 2, (6, 6), (3, 3)
    z = RNG.standard_normal((N, K) + grid) * (RNG.random((N, K) + grid) < 0.5)
    b = RNG.standard_normal((N, 1) + grid)
    mu = np.array([0.7, 1.9])
    d_ref, W = learning_dense(b[:, 0], z, fs, mu)
    d, mu_out, gamma = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=300)
    nrm = np.sqrt((d_ref.reshape(K, -1) ** 2).sum(1))
    want = d_ref / np.maximum(1.0, nrm).reshape(K, 1, 1)
    np.testing.assert_allclose(d[:, 0], want, atol=1e-12)
    np.testing.assert_allclose(mu_out, mu * nrm, rtol=1e-12)
    # gamma* = Z S^T d* - x
    np.testing.assert_allclose(gamma[:, 0].reshape(-1), W @ d_ref.reshape(-1) - b[:, 0].reshape(-1),
                               atol=1e-11)


def test_learning_tensor_separates_over_channels():
    N, K, J, grid, fs = 2, 2, 3, (6, 6), (3, 3)
    z = RNG.standard_normal((N, K) + grid) * (RNG.random((N, K) + grid) < 0.5)
    b = RNG.standard_normal((N, J) + grid)
    mu = np.array([1.3, 0.8])
    d, mu_out, _ = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=300)
    ref = np.stack([learning_dense(b[:, j], z, fs, mu)[0] for j in range(J)], axis=1)
    nrm = np.sqrt((ref.reshape(K, -1) ** 2).sum(1))        # norm over channels and taps
    np.testing.assert_allclose(d, ref / np.maximum(1.0, nrm).reshape(K, 1, 1, 1), atol=1e-12)
    np.testing.assert_allclose(mu_out, mu * nrm, rtol=1e-12)


def test_cg_fixed_count_matches_dense_steps():
    """A few CG iterations agree with CG on the dense operator
    I + sum_k W_k W_k^T / (2 mu_k)."""
    N, K, grid, fs = 2, 2, (6, 6), (3, 3)
    z = RNG.standard_normal((N, K) + grid) * (RNG.random((N, K) + grid) < 0.5)
    b = RNG.standard_normal((N, 1) + grid)
    mu = np.array([0.9, 1.1])
    _, W = learning_dense(b[:, 0], z, fs, mu)
    M = int(np.prod(fs))
    A = np.eye(W.shape[0]) + (W / np.repeat(2 * mu, M)) @ W.T
    x = np.zeros(W.shape[0])
    rhs = -b[:, 0].reshape(-1)
    r = rhs - A @ x
    p = r.copy()
    rr = r @ r
    for _ in range(4):
        ap = A @ p
        al = rr / (p @ ap)
        x += al * p
        r -= al * ap
        rn = r @ r
        p = r + rn / rr * p
        rr = rn
    _, _, gamma = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=4)
    np.testing.assert_allclose(gamma[:, 0].reshape(-1), x, atol=1e-12)


def test_mu_iteration_fixed_point_unit_norm():
    """eq:mu_update: with the constraint active (codes small next to the
    images, so the unregularised filters would be long) ||d_k|| -> 1 and mu is
    a fixed point; with it inactive mu -> 0 and ||d_k|| < 1 (complementary
    slackness)."""
    N, K, grid, fs = 2, 3, (12, 12), (4, 4)
    rng = np.random.default_rng(3)  # own generator: the result must not depend on test order
    mask = rng.random((N, K) + grid) < 0.3
    z = rng.standard_normal((N, K) + grid) * mask * 0.3
    b = rng.standard_normal((N, 1) + grid) * 3
    d, mu, _ = oracle.learn(b, z, fs, np.ones(K), None, inner_iters=80, cg_iters=200)
    nrm = np.sqrt((d.reshape(K, -1) ** 2).sum(1))
    np.testing.assert_allclose(nrm, 1.0, atol=1e-6)
    d2, mu2, _ = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=200)
    np.testing.assert_allclose(mu2, mu, rtol=1e-6)
    # inactive: codes large, so the least-squares filters are short.  mu
    # falls geometrically here (1e-13 within 10 updates), after which the
    # system of eq:Learning_gamma is too ill-conditioned for CG to keep
    # ||d_k|| below 1, so the check stops at 10 updates
    d3, mu3, _ = oracle.learn(b, z * 100, fs, np.ones(K), None, inner_iters=10, cg_iters=200)
    nrm3 = np.sqrt((d3.reshape(K, -1) ** 2).sum(1))
    assert np.all(nrm3 < 1.0) and np.all(mu3 < 1e-3)


def test_zero_filter_keeps_multiplier():
    N, K, grid, fs = 2, 2, (8, 8), (3, 3)
    z = RNG.standard_normal((N, K) + grid)
    z[:, 1] = 0.0
    b = RNG.standard_normal((N, 1) + grid)
    d, mu, _ = oracle.learn(b, z, fs, np.array([1.0, 2.5]), None, inner_iters=3, cg_iters=20)
    assert mu[1] == 2.5 and np.all(d[1] == 0) and np.all(np.isfinite(d))


# ---------------------------------------------------------- P12 alternation

def test_alternation_monotone_with_tight_inner_solves():
    grid, fs, K = (16, 16), (5, 5), 4
    b = RNG.standard_normal((2, 1) + grid) * 3
    d0 = rand_filters(K, 1, fs)
    d, z, th, mu, gamma = d0, None, None, np.ones(K), None
    objs = []
    for _ in range(4):
        out = oracle.code(b, d, 0.5, 1.0, 1500, z0=z, theta0=th)
        z, th = out["z"], out["theta"]
        objs.append(oracle.objective(b, d, z, 0.5)[1])
        d, mu, gamma = oracle.learn(b, z, fs, mu, gamma, inner_iters=60, cg_iters=150)
        objs.append(oracle.objective(b, d, z, 0.5)[1])
    assert all(o2 <= o1 * (1 + 1e-7) for o1, o2 in zip(objs, objs[1:])), objs
    assert objs[-1] < objs[0]


def _alg1_by_hand(b, d0, beta, rho, t_in, t_out, inner, cg, cold=False, reset_mu=False, reset_rho=False):
    """Alg. 1 written out from its description: z, theta start at zero, mu at
    1, gamma at 0, rho at its initial value, all set once before the loop and
    carried from one outer step to the next (coding warm-starts from the
    previous codes and split variable, learning from the previous gamma and
    multipliers).  The flags plant the mistakes the pin must catch."""
    K = d0.shape[0]
    d, z, th, mu, gamma = np.asarray(d0, float), None, None, np.ones(K), None
    rho_v = np.full(b.shape[0], float(rho))
    objs = []
    for _ in range(t_out):
        if cold:
            z = th = None
        if reset_mu:
            mu, gamma = np.ones(K), None
        if reset_rho:
            rho_v = np.full(b.shape[0], float(rho))
        out = oracle.code(b, d, beta, rho_v, t_in, z0=z, theta0=th, adaptive=True)
        z, th, rho_v = out["z"], out["theta"], out["rho"][-1]
        objs.append(oracle.objective(b, d, z, beta)[1])
        d, mu, gamma = oracle.learn(b, z, d0.shape[2:], mu, gamma, inner, cg)
        objs.append(oracle.objective(b, d, z, beta)[1])
    return d, z, th, mu, gamma, objs


def test_learn_dictionary_is_alg1_with_carried_state():
    """learn_dictionary equals Alg. 1 written out by hand (3 outer steps,
    adaptive rho) bit for bit, and each planted mistake -- a cold restart of
    z and theta, a reset of mu and gamma, a reset of rho -- moves the result
    far beyond rounding, so any of them inside learn_dictionary fails here."""
    grid, fs, K = (16, 16), (5, 5), 4
    rng = np.random.default_rng(12)
    b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, grid))[None] * 10 for _ in range(2)])
    d0 = rand_filters(K, 1, fs, rng)
    out = oracle.learn_dictionary(b, d0, 1.0, 10.0, 6, 3, 3, 4, adaptive=True)
    d, z, th, mu, gamma, objs = _alg1_by_hand(b, d0, 1.0, 10.0, 6, 3, 3, 4)
    assert np.count_nonzero(z) / z.size > 0.01
    for got, want in ((out["d"], d), (out["z"], z), (out["theta"], th), (out["mu"], mu), (out["gamma"], gamma)):
        assert np.array_equal(got, want)
    assert out["objectives"] == objs
    for mistake in ("cold", "reset_mu", "reset_rho"):
        bad = _alg1_by_hand(b, d0, 1.0, 10.0, 6, 3, 3, 4, **{mistake: True})
        assert np.abs(bad[0] - d).max() > 1e-6 or np.abs(bad[1] - z).max() > 1e-6, mistake


def test_learn_dictionary_monotone_with_tight_inner_solves():
    """P12 through learn_dictionary itself: with tight inner solves (1500
    coding iterations, 60 multiplier updates of 150 CG steps) and the final
    projection into the unit ball, the objective does not increase across
    half steps."""
    grid, fs, K = (16, 16), (5, 5), 4
    rng = np.random.default_rng(21)
    b = rng.standard_normal((2, 1) + grid) * 3
    d0 = rand_filters(K, 1, fs, rng)
    out = oracle.learn_dictionary(b, d0, 0.5, 1.0, 1500, 3, 60, 150)
    objs = out["objectives"]
    assert all(o2 <= o1 * (1 + 1e-7) for o1, o2 in zip(objs, objs[1:])), objs
    assert objs[-1] < objs[0]


def test_learn_dictionary_runs_and_logs():
    grid, fs, K = (12, 12), (3, 3), 3
    b = RNG.standard_normal((2, 1) + grid) * 3
    out = oracle.learn_dictionary(b, rand_filters(K, 1, fs), 0.5, 1.0, 5, 2, 3, 5)
    assert len(out["objectives"]) == 4
    assert np.all(np.sqrt((out["d"].reshape(K, -1) ** 2).sum(1)) <= 1 + 1e-12)


# --------------------------------------------------------------- P14 gradient

def _fd_margin_ok(b, d, beta, rho, T, margin):
    """Every clip argument stays at least ``margin`` away from +-beta."""
    N, J = b.shape[:2]
    grid = b.shape[2:]
    K = d.shape[0]
    Dm = dict_matrix(d, grid)
    A = Dm @ Dm.T + np.eye(Dm.shape[0]) / rho
    for n in range(N):
        x = b[n].reshape(-1)
        z = np.zeros(Dm.shape[1])
        th = np.zeros_like(z)
        for _ in range(T):
            lam = np.linalg.solve(A, Dm @ th + Dm @ z / rho - x / rho)
            v = Dm.T @ lam
            u = v - z / rho
            if np.min(np.abs(np.abs(u) - beta)) < margin:
                return False
            th = np.clip(u, -beta, beta)
            z = z + rho * (th - v)
    return True


def test_gradient_matches_finite_differences():
    """Oracle reverse pass vs FP64 central differences on a small instance
    (2 images 16x16, K = 3, 5x5 taps, 30 iterations)."""
    rng = np.random.default_rng(7)
    grid, fs, K, T, rho, beta = (10, 10), (3, 3), 3, 30, 10.0, 1.0
    b = rng.standard_normal((2, 1) + grid) * 10
    d = rand_filters(K, 1, fs, rng)
    assert _fd_margin_ok(b, d, beta, rho, T, 1e-6)
    L, gd, gb = oracle.code_loss_grad(b, d, beta, rho, T)
    z = oracle.code(b, d, beta, rho, T)["z"]
    assert abs(L - oracle.objective(b, d, z, beta)[1]) < 1e-10 * abs(L)
    assert np.count_nonzero(z) > 0

    def loss(dd, bb):
        zz = oracle.code(b, dd, bb, rho, T)["z"]
        return oracle.objective(b, dd, zz, bb)[1]

    h = 1e-6
    scale = max(np.abs(gd).max(), abs(gb))
    picks = list(itertools.product(range(K), range(fs[0]), range(fs[1])))
    for (k, m0, m1) in picks:
        dp = d.copy(); dp[k, 0, m0, m1] += h
        dm = d.copy(); dm[k, 0, m0, m1] -= h
        fd = (loss(dp, beta) - loss(dm, beta)) / (2 * h)
        assert abs(fd - gd[k, 0, m0, m1]) <= 1e-6 * scale, (k, m0, m1, fd, gd[k, 0, m0, m1])
    fd_b = (loss(d, beta + h) - loss(d, beta - h)) / (2 * h)
    assert abs(fd_b - gb) <= 1e-6 * scale


def test_gradient_tensor_matches_finite_differences():
    rng = np.random.default_rng(11)
    grid, fs, K, J, T, rho, beta = (8, 8), (3, 3), 2, 2, 10, 3.0, 0.5
    b = rng.standard_normal((1, J) + grid) * 4
    d = rand_filters(K, J, fs, rng)
    assert _fd_margin_ok(b, d, beta, rho, T, 1e-6)
    L, gd, gb = oracle.code_loss_grad(b, d, beta, rho, T)

    def loss(dd, bb):
        zz = oracle.code(b, dd, bb, rho, T)["z"]
        return oracle.objective(b, dd, zz, bb)[1]

    h = 1e-6
    scale = max(np.abs(gd).max(), abs(gb))
    for idx in [(0, 0, 0, 0), (1, 1, 2, 1), (0, 1, 1, 2), (1, 0, 2, 2)]:
        dp = d.copy(); dp[idx] += h
        dm = d.copy(); dm[idx] -= h
        fd = (loss(dp, beta) - loss(dm, beta)) / (2 * h)
        assert abs(fd - gd[idx]) <= 1e-6 * scale
    fd_b = (loss(d, beta + h) - loss(d, beta - h)) / (2 * h)
    assert abs(fd_b - gb) <= 1e-6 * scale


def test_objective_grad_finite_differences():
    rng = np.random.default_rng(3)
    grid, fs, K, J = (8, 8), (3, 3), 3, 2
    d = rand_filters(K, J, fs, rng)
    z = rng.standard_normal((2, K) + grid) * (rng.random((2, K) + grid) < 0.4)
    b = rng.standard_normal((2, J) + grid)
    beta = 0.6
    f, dz, dd, db = oracle.objective_grad(b, d, z, beta)
    assert abs(f - oracle.objective(b, d, z, beta)[1]) < 1e-12 * abs(f)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 2, 1), (2, 0, 1, 2)]:
        dp = d.copy(); dp[idx] += h
        dm = d.copy(); dm[idx] -= h
        fd = (oracle.objective(b, dp, z, beta)[1] - oracle.objective(b, dm, z, beta)[1]) / (2 * h)
        assert abs(fd - dd[idx]) < 1e-6 * max(1.0, abs(fd))
    nz = np.argwhere(z != 0)
    for idx in [tuple(nz[0]), tuple(nz[5])]:
        zp = z.copy(); zp[idx] += h
        zm = z.copy(); zm[idx] -= h
        fd = (oracle.objective(b, d, zp, beta)[1] - oracle.objective(b, d, zm, beta)[1]) / (2 * h)
        assert abs(fd - dz[idx]) < 1e-6 * max(1.0, abs(fd))
    assert db == np.abs(z).sum()


@pytest.mark.slow
def test_gradient_fd_on_unrolled_instance():
    """The unrolled-coding FD instance (2 x 32x32 images, K = 4 11x11 filters,
    30 iterations, rho = 10, beta = 1): oracle reverse pass vs FP64 central
    differences on a subset of taps and beta."""
    import synth
    cfg = synth.CONFIGS["unrolled_fd"]
    b, d = synth.make_inputs(cfg)
    b = b.astype(np.float64)
    d = d.astype(np.float64)
    # every clip argument keeps a margin far above the FD perturbation
    from oracle.csc import _dual_solve, _fft, _gram, _ifft_real, filter_spectra
    dh = filter_spectra(d, b.shape[2:])
    G = _gram(dh)
    xh = _fft(b, 2)
    z = np.zeros((b.shape[0], cfg.k) + b.shape[2:])
    th = np.zeros_like(z)
    margin = np.inf
    for _ in range(cfg.t_in):
        rhs = np.einsum("jk...,nk...->nj...", dh, _fft(th + z / cfg.rho, 2)) - xh / cfg.rho
        lam = _dual_solve(G, rhs, np.full(b.shape[0], cfg.rho))
        v = _ifft_real(np.einsum("jk...,nj...->nk...", np.conj(dh), lam), 2)
        u = v - z / cfg.rho
        margin = min(margin, np.min(np.abs(np.abs(u) - cfg.beta)))
        th = np.clip(u, -cfg.beta, cfg.beta)
        z = z + cfg.rho * (th - v)
    assert margin > 1e-6
    L, gd, gb = oracle.code_loss_grad(b, d, cfg.beta, cfg.rho, cfg.t_in)

    def loss(dd, bb):
        zz = oracle.code(b, dd, bb, cfg.rho, cfg.t_in)["z"]
        return oracle.objective(b, dd, zz, bb)[1]

    h = 1e-7
    scale = max(np.abs(gd).max(), abs(gb))
    rng = np.random.default_rng(0)
    for _ in range(10):
        idx = (int(rng.integers(cfg.k)), 0, int(rng.integers(11)), int(rng.integers(11)))
        dp = d.copy(); dp[idx] += h
        dm = d.copy(); dm[idx] -= h
        fd = (loss(dp, cfg.beta) - loss(dm, cfg.beta)) / (2 * h)
        assert abs(fd - gd[idx]) <= 1e-6 * scale, (idx, fd, gd[idx])
    fd_b = (loss(d, cfg.beta + h) - loss(d, cfg.beta - h)) / (2 * h)
    assert abs(fd_b - gb) <= 1e-6 * scale


# ------------------------------------------- convergence-driven stopping rules

def test_code_tolerance_stops_at_first_iteration_meeting_the_rule():
    """The tolerance mode stops after the first iteration at which every
    image's RMS primal and dual residuals are at most tol (read off the
    residual history of a fixed-count run), with the same iterates as that
    run truncated there; a huge tol stops after one iteration and a zero-like
    tol never fires."""
    rng = np.random.default_rng(71)
    b = rng.standard_normal((2, 1, 16, 16)) * 3
    d = rand_filters(3, 1, (3, 3), rng)
    K, J, npix = 3, 1, 256
    full = oracle.code(b, d, 0.5, 2.0, 40)
    rms = np.maximum(full["resid"][:, :, 0] / np.sqrt(K * npix), full["resid"][:, :, 1] / np.sqrt(J * npix))
    worst = rms.max(axis=1)                       # [iters]: the largest RMS residual over images and kinds
    k = 12
    tol = float(np.sqrt(worst[k] * worst[:k].min())) if worst[:k].min() > worst[k] else None
    assert tol is not None and worst[k] <= tol < worst[:k].min()
    first = int(np.argmax(worst <= tol))
    got = oracle.code(b, d, 0.5, 2.0, 40, tol=tol)
    assert got["iters"] == first + 1
    trunc = oracle.code(b, d, 0.5, 2.0, first + 1)
    np.testing.assert_array_equal(got["z"], trunc["z"])
    np.testing.assert_array_equal(got["resid"], full["resid"][:first + 1])
    assert oracle.code(b, d, 0.5, 2.0, 40, tol=1e9)["iters"] == 1
    assert oracle.code(b, d, 0.5, 2.0, 7, tol=1e-300)["iters"] == 7


def test_cg_tolerance_meets_the_rule_minimally_on_the_dense_operator():
    """With cg_tol the CG solve of eq:Learning_gamma stops at the first step
    whose residual, measured on the dense operator I + sum_k W_k W_k^T /
    (2 mu_k), is at most cg_tol ||x||: the step before does not meet it."""
    N, K, grid, fs = 2, 2, (6, 6), (3, 3)
    rng = np.random.default_rng(72)
    z = rng.standard_normal((N, K) + grid) * (rng.random((N, K) + grid) < 0.5)
    b = rng.standard_normal((N, 1) + grid)
    mu = np.array([0.9, 1.1])
    _, W = learning_dense(b[:, 0], z, fs, mu)
    M = int(np.prod(fs))
    A = np.eye(W.shape[0]) + (W / np.repeat(2 * mu, M)) @ W.T
    x = b[:, 0].reshape(-1)
    tol = 1e-4
    info = {}
    _, _, g = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=200, cg_tol=tol, info=info)
    steps = info["cg_counts"][0]
    assert 0 < steps < 200
    res = np.linalg.norm(-x - A @ g[:, 0].reshape(-1))
    assert res <= tol * np.linalg.norm(x) * (1 + 1e-9)
    _, _, g1 = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=steps - 1)
    assert np.linalg.norm(-x - A @ g1[:, 0].reshape(-1)) > tol * np.linalg.norm(x)
    _, _, g2 = oracle.learn(b, z, fs, mu, None, inner_iters=1, cg_iters=steps)
    np.testing.assert_array_equal(g2, g)


def test_cg_tolerance_warm_start_needs_fewer_steps():
    """Warm-started solves (gamma carried across multiplier updates, Sec.
    3.2.2) reach the tolerance in fewer CG steps than the first, cold one."""
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg, n=2)
    z = oracle.code(b, d, cfg.beta, cfg.rho, 10)["z"]
    info = {}
    oracle.learn(b, z, cfg.fsupp, np.ones(cfg.k), None, inner_iters=6, cg_iters=50, cg_tol=1e-3, info=info)
    c = info["cg_counts"]
    assert c[0] > max(c[2:]), c


def test_alternation_tau_stops_on_the_objective_change():
    """learn_dictionary with tau ends after the first outer step whose
    objective (after learning) changed by at most tau relative to the
    previous step's; no earlier step met that."""
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg, n=2)
    tau = 0.05
    out = oracle.learn_dictionary(b, d0, cfg.beta, cfg.rho, 5, 12, 3, 5, tau=tau)
    f = np.array(out["objectives"][1::2])              # after each learning half step
    assert len(f) == out["steps"]
    rel = np.abs(np.diff(f)) / np.abs(f[:-1])
    if out["steps"] < 12:
        assert rel[-1] <= tau and np.all(rel[:-1] > tau)
    else:
        assert np.all(rel > tau)
    full = oracle.learn_dictionary(b, d0, cfg.beta, cfg.rho, 5, out["steps"], 3, 5)
    np.testing.assert_array_equal(full["d"], out["d"])
