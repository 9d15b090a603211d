"""Pins for the oracle's nuclear-norm regulariser (Sec. 5: a nuclear norm on
the sparse maps makes them low rank).  The coding problem becomes
min_z 1/2 ||x - sum_k d_k * z_k||^2 + beta sum_k ||z_k||_*, whose dual ADMM
(eq:Inference_solution) keeps every update except the projection Pi_C, now
onto the beta-ball of the spectral norm (the dual norm of the nuclear norm).

The reference values here are built another way than the oracle's SVD
route: spectral projections and thresholds from the eigen-decomposition of
u^T u, dense convolution matrices from test_oracle.py, closed forms."""
import numpy as np
import pytest

import oracle
from test_oracle import dict_matrix, rand_filters


def eig_route(u, beta, mode):
    """Projection onto ||.||_2 <= beta (mode "proj") or singular value
    thresholding at beta (mode "svt") of one matrix, from u^T u = V diag(s^2) V^T:
    u V diag(f(s)) V^T with f(s) = min(1, beta/s) or max(0, 1 - beta/s)."""
    s2, V = np.linalg.eigh(u.T @ u)
    s = np.sqrt(np.maximum(s2, 0.0))
    with np.errstate(divide="ignore"):
        f = np.minimum(1.0, beta / s) if mode == "proj" else np.maximum(0.0, 1.0 - beta / s)
    f = np.where(s > 0, f, 1.0 if mode == "proj" else 0.0)
    return u @ V @ np.diag(f) @ V.T


def test_diagonal_matrix_projection_is_a_clip():
    """For a diagonal matrix the singular values are |diag|, so the spectral
    projection is the l-infinity clip of the diagonal and SVT is soft."""
    rng = np.random.default_rng(1)
    dg = rng.standard_normal(9) * 2
    P = oracle.project_spectral_ball(np.diag(dg), 0.7)
    np.testing.assert_allclose(P, np.diag(np.clip(dg, -0.7, 0.7)), atol=1e-13)
    np.testing.assert_allclose(oracle.svt(np.diag(dg), 0.7), np.diag(oracle.soft(dg, 0.7)), atol=1e-13)
    np.testing.assert_allclose(oracle.nuclear_norm(np.diag(dg)), np.abs(dg).sum(), rtol=1e-13)


@pytest.mark.parametrize("shape", [(8, 8), (12, 6), (5, 10)])
def test_projection_and_svt_against_eigen_route(shape):
    rng = np.random.default_rng(2)
    u = rng.standard_normal(shape) * 3
    beta = 2.5
    np.testing.assert_allclose(oracle.project_spectral_ball(u, beta), eig_route(u, beta, "proj"), atol=1e-10)
    np.testing.assert_allclose(oracle.svt(u, beta), eig_route(u, beta, "svt"), atol=1e-10)
    # nuclear norm as the trace of (u^T u)^(1/2)
    s2 = np.linalg.eigvalsh(u.T @ u if shape[0] >= shape[1] else u @ u.T)
    np.testing.assert_allclose(oracle.nuclear_norm(u), np.sqrt(np.maximum(s2, 0)).sum(), rtol=1e-12)


def test_projection_variational_inequality():
    """P = Pi_C(u) is feasible and <u - P, Q - P> <= 0 for every feasible Q;
    points of C are fixed."""
    rng = np.random.default_rng(3)
    beta = 1.5
    u = rng.standard_normal((10, 10)) * 2
    P = oracle.project_spectral_ball(u, beta)
    assert np.linalg.norm(P, 2) <= beta * (1 + 1e-12)
    for _ in range(200):
        Q = rng.standard_normal((10, 10))
        Q *= beta * rng.random() / np.linalg.norm(Q, 2)
        assert np.sum((u - P) * (Q - P)) <= 1e-10
    inside = u * (0.9 * beta / np.linalg.norm(u, 2))
    np.testing.assert_allclose(oracle.project_spectral_ball(inside, beta), inside, atol=1e-12)


def test_svt_is_the_proximal_operator():
    """p = svt(u, t) minimises 1/2 ||x - u||^2 + t ||x||_*: no random nearby
    point does better, and (u - p)/t = U1 V1^T + W with W orthogonal to p's
    singular spaces and ||W||_2 <= 1."""
    rng = np.random.default_rng(4)
    u = rng.standard_normal((8, 8)) * 2
    t = 1.2
    p = oracle.svt(u, t)

    def h(x):
        return 0.5 * np.sum((x - u) ** 2) + t * np.linalg.svd(x, compute_uv=False).sum()

    hp = h(p)
    for _ in range(300):
        assert h(p + 1e-3 * rng.standard_normal(p.shape)) >= hp - 1e-12
    U, s, Vt = np.linalg.svd(p)
    r = int((s > 1e-9).sum())
    assert 0 < r < 8
    g = (u - p) / t
    U1, V1 = U[:, :r], Vt[:r].T
    np.testing.assert_allclose(U1.T @ g @ V1, np.eye(r), atol=1e-10)
    W = g - U1 @ V1.T
    np.testing.assert_allclose(U1.T @ W, 0, atol=1e-10)
    np.testing.assert_allclose(W @ V1, 0, atol=1e-10)
    assert np.linalg.norm(W, 2) <= 1 + 1e-10


def dense_admm_nuclear(x, Dm, grid, K, beta, rho, iters):
    """eq:Inference_solution with dense matrices and the spectral-ball
    projection per map (eigen route)."""
    KD = Dm.shape[1]
    z = np.zeros(KD)
    th = np.zeros(KD)
    A = Dm @ Dm.T + np.eye(Dm.shape[0]) / rho
    for _ in range(iters):
        lam = np.linalg.solve(A, Dm @ th + Dm @ z / rho - x / rho)
        v = Dm.T @ lam
        u = (v - z / rho).reshape((K,) + grid)
        th_new = np.stack([eig_route(u[k], beta, "proj") for k in range(K)]).reshape(-1)
        z = z + rho * (th_new - v)
        th = th_new
    return z.reshape((K,) + grid), th.reshape((K,) + grid)


@pytest.mark.parametrize("J", [1, 2])
def test_nuclear_coding_matches_dense_admm(J):
    rng = np.random.default_rng(5)
    grid, fs, K = (8, 10), (3, 3), 3
    d = rand_filters(K, J, fs, rng)
    b = rng.standard_normal((1, J) + grid) * 3
    out = oracle.code(b, d, 0.9, 2.0, 25, reg="nuclear")
    z, th = dense_admm_nuclear(b[0].reshape(-1), dict_matrix(d, grid), grid, K, 0.9, 2.0, 25)
    np.testing.assert_allclose(out["z"][0], z, atol=1e-10)
    np.testing.assert_allclose(out["theta"][0], th, atol=1e-10)
    ranks = [np.linalg.matrix_rank(z[k], tol=1e-8) for k in range(K)]
    assert 0 < min(ranks) and max(ranks) < min(grid)


def test_nuclear_delta_filter_gives_svt():
    """K = 1 with a delta filter: min 1/2 ||x - z||^2 + beta ||z||_* is solved
    by singular value thresholding of x."""
    rng = np.random.default_rng(6)
    grid = (12, 12)
    d = np.zeros((1, 1, 3, 3))
    d[0, 0, 0, 0] = 1.0
    b = rng.standard_normal((2, 1) + grid) * 2
    out = oracle.code(b, d, 2.0, 2.0, 300, reg="nuclear")
    for n in range(2):
        np.testing.assert_allclose(out["z"][n, 0], eig_route(b[n, 0], 2.0, "svt"), atol=1e-10)


def test_nuclear_kkt_and_duality_gap_at_convergence():
    """At the solution g_k = D_k^T (x - D z) lies in beta times the
    subdifferential of the nuclear norm at z_k, and the primal objective
    equals the dual max_{||D^T lam||_2 <= beta} -1/2 ||lam||^2 - <lam, x>
    at lam = D z - x."""
    rng = np.random.default_rng(7)
    grid, fs, K, beta = (12, 12), (4, 4), 3, 1.0
    d = rand_filters(K, 1, fs, rng)
    b = rng.standard_normal((1, 1) + grid) * 3
    out = oracle.code(b, d, beta, 1.0, 4000, reg="nuclear")
    z = out["z"][0]
    Dm = dict_matrix(d, grid)
    res = b[0, 0].reshape(-1) - Dm @ z.reshape(-1)
    g = (Dm.T @ res).reshape(z.shape)
    for k in range(K):
        U, s, Vt = np.linalg.svd(z[k])
        r = int((s > 1e-7 * max(1.0, s[0])).sum())
        assert np.linalg.norm(g[k], 2) <= beta * (1 + 1e-6)
        if r:
            U1, V1 = U[:, :r], Vt[:r].T
            np.testing.assert_allclose(U1.T @ g[k] @ V1, beta * np.eye(r), atol=1e-6)
    primal = 0.5 * res @ res + beta * sum(np.linalg.svd(z[k], compute_uv=False).sum() for k in range(K))
    lam = -res
    scale = min(1.0, beta / max(np.linalg.norm((Dm.T @ lam).reshape(z.shape)[k], 2) for k in range(K)))
    lam = lam * scale
    dual = -0.5 * lam @ lam - lam @ b[0, 0].reshape(-1)
    assert 0 <= primal - dual <= 1e-7 * abs(primal)
    np.testing.assert_allclose(oracle.objective(b, d, out["z"], beta, reg="nuclear")[1], primal, rtol=1e-12)
