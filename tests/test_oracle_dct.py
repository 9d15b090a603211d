"""Pins for the oracle of the DCT-domain variant (symmetric boundaries,
oracle/dct.py): each check compares it with something built another way --
dense matrices of the symmetric-boundary convolution filled tap by tap with
explicit reflections, the circular oracle run on the symmetric extension of
the image, closed forms and optimality conditions."""
import numpy as np
import pytest

import oracle
from oracle import dct
from test_oracle import dense_admm


def reflect(i, n):
    """Index of the half-sample symmetric extension of a length-n axis."""
    i = i % (2 * n)
    return i if i < n else 2 * n - 1 - i


def sym_conv_matrix(q, grid):
    """Dense D x D matrix of z -> sum_m h[m] z~[p - m], h the symmetric
    filter of quadrant q, z~ the half-sample symmetric extension of z."""
    H, W = grid
    M1, M2 = q.shape
    A = np.zeros((H * W, H * W))
    for p1 in range(H):
        for p2 in range(W):
            for m1 in range(-M1 + 1, M1):
                for m2 in range(-M2 + 1, M2):
                    s1, s2 = reflect(p1 - m1, H), reflect(p2 - m2, W)
                    A[p1 * W + p2, s1 * W + s2] += q[abs(m1), abs(m2)]
    return A


def sym_dict_matrix(q, grid):
    K, J = q.shape[:2]
    return np.vstack([np.hstack([sym_conv_matrix(q[k, j], grid) for k in range(K)]) for j in range(J)])


def rand_q(K, J, M, rng):
    q = rng.standard_normal((K, J) + M)
    f = dct.full_filter(q)
    return q / np.sqrt((f.reshape(K, -1) ** 2).sum(1)).reshape(K, 1, 1, 1)


@pytest.mark.parametrize("grid,M,J", [((6, 5), (3, 2), 1), ((8, 8), (4, 4), 2), ((7, 9), (1, 3), 1)])
def test_symmetric_convolution_bruteforce(grid, M, J):
    rng = np.random.default_rng(1)
    K = 3
    q = rand_q(K, J, M, rng)
    z = rng.standard_normal((2, K) + grid)
    Dm = sym_dict_matrix(q, grid)
    got = dct.reconstruct(q, z)
    for n in range(2):
        np.testing.assert_allclose(got[n].reshape(-1), Dm @ z[n].reshape(-1), atol=1e-12)
    # the operator of each filter is symmetric: D_k^T = D_k
    for k in range(K):
        A = sym_conv_matrix(q[k, 0], grid)
        np.testing.assert_allclose(A, A.T, atol=1e-13)


def test_full_filter_is_the_quadrant_mirrored():
    q = np.arange(6.0).reshape(2, 3)
    f = dct.full_filter(q)
    assert f.shape == (3, 5)
    for a in range(-1, 2):
        for c in range(-2, 3):
            assert f[a + 1, c + 2] == q[abs(a), abs(c)]


@pytest.mark.parametrize("J", [1, 2])
def test_dct_coding_matches_dense_admm(J):
    rng = np.random.default_rng(2)
    grid, M, K = (8, 6), (3, 3), 3
    q = rand_q(K, J, M, rng)
    b = rng.standard_normal((1, J) + grid) * 3
    out = dct.code(b, q, 0.7, 2.0, 20)
    z, th, _ = dense_admm(b[0].reshape(-1), sym_dict_matrix(q, grid), 0.7, 2.0, 20)
    np.testing.assert_allclose(out["z"][0].reshape(-1), z, atol=1e-10)
    np.testing.assert_allclose(out["theta"][0].reshape(-1), th, atol=1e-10)
    assert 0.02 < np.count_nonzero(z) / z.size < 0.9


def test_dct_coding_equals_circular_coding_of_the_symmetric_extension():
    """The circular oracle run on the 2H x 2W half-sample symmetric extension
    of the image, with the full symmetric filter (corner anchored, so its
    codes come out shifted by M - 1), takes the same iterates: its codes are
    the symmetric extension of the DCT variant's (same beta and rho)."""
    rng = np.random.default_rng(3)
    H, W, M, K = 8, 6, (3, 2), 2
    q = rand_q(K, 1, M, rng)
    b = rng.standard_normal((1, 1, H, W)) * 3
    ext = np.concatenate([b, b[..., ::-1, :]], axis=-2)
    ext = np.concatenate([ext, ext[..., :, ::-1]], axis=-1)          # [1][1][2H][2W]
    out_c = oracle.code(ext, dct.full_filter(q), 0.8, 2.0, 25)
    out_s = dct.code(b, q, 0.8, 2.0, 25)
    zc = np.roll(out_c["z"], shift=(M[0] - 1, M[1] - 1), axis=(-2, -1))
    np.testing.assert_allclose(zc[..., :H, :W], out_s["z"], atol=1e-10)
    np.testing.assert_allclose(zc[..., H:, :W], out_s["z"][..., ::-1, :], atol=1e-10)
    assert np.count_nonzero(out_s["z"]) > 0


def test_dct_delta_filter_gives_soft_threshold():
    rng = np.random.default_rng(4)
    q = np.zeros((1, 1, 2, 2))
    q[0, 0, 0, 0] = 1.0
    b = rng.standard_normal((2, 1, 10, 12)) * 2
    out = dct.code(b, q, 0.8, 2.0, 200)
    np.testing.assert_allclose(out["z"][:, 0], oracle.soft(b[:, 0], 0.8), atol=1e-12)


def test_dct_kkt_at_convergence():
    rng = np.random.default_rng(5)
    grid, M, K, beta = (10, 10), (3, 3), 3, 1.0
    q = rand_q(K, 1, M, rng)
    b = rng.standard_normal((1, 1) + grid) * 3
    out = dct.code(b, q, beta, 1.0, 3000)
    z = out["z"][0]
    Dm = sym_dict_matrix(q, grid)
    g = (Dm.T @ (b[0, 0].reshape(-1) - Dm @ z.reshape(-1))).reshape(z.shape)
    on = z != 0
    assert on.sum() > 0
    np.testing.assert_allclose(g[on], beta * np.sign(z[on]), atol=1e-8)
    assert np.abs(g[~on]).max() <= beta + 1e-8
    per, tot = dct.objective(b, q, out["z"], beta)
    res = b[0, 0].reshape(-1) - Dm @ z.reshape(-1)
    np.testing.assert_allclose(tot, 0.5 * res @ res + beta * np.abs(z).sum(), rtol=1e-12)
