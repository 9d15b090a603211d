"""Degenerate shapes on the GPU against the FP64 oracle: a single filter
(K = 1, one half-empty pair), a support as large as the grid, a 1 x 1
support, non-square supports, N = 1, and the smallest grids of the learning
path (one pass-A workgroup covering every canonical row).  Tolerances as in
test_gpu_parity.py (codes 1e-4, or 3e-6 max|z| for large codes; filters
1e-4 of max(1, max|d|)).  With a 1 x 1 unit filter the coding problem
separates per pixel, and after enough iterations the codes approach the
soft threshold of the image, the closed form of the lasso with an identity
dictionary."""
import numpy as np
import pytest

import oracle
import synth
from tolerances import CODE_TOL, code_tol

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)




def case(seed, n, j, k, grid, fsupp, amp=10.0):
    rng = np.random.default_rng(seed)
    b = np.zeros((n, j) + grid, np.float32)
    for i in range(n):
        for c in range(j):
            b[i, c] = synth.contrast_normalize(synth.one_over_f(rng, grid)) * amp
    return b, synth.unit_filters(k, j, fsupp, seed + 1)


@pytest.mark.parametrize("grid,k,fs,n", [
    ((64, 64), 1, (11, 11), 2),     # one filter: a single half-empty pair
    ((16, 16), 3, (16, 16), 2),     # support as large as the grid
    ((32, 32), 4, (1, 1), 1),       # 1 x 1 support
    ((64, 128), 5, (5, 11), 1),     # non-square support on a rectangular grid
    ((256, 256), 1, (3, 7), 1),     # split path, K = 1, non-square support
])
def test_code_degenerate_shapes(lib, grid, k, fs, n):
    b, d = case(81 + k, n, 1, k, grid, fs)
    ref = oracle.code(b, d, 1.0, 5.0, 12)
    z = N(lib.code(T(b), T(d), 1.0, 5.0, 12)[0])
    assert np.count_nonzero(ref["z"]) > 0
    assert np.abs(z - ref["z"]).max() <= code_tol(ref["z"])


def test_code_identity_dictionary_soft_threshold(lib):
    """K = 1, d = [1] (1 x 1): z -> soft(x, beta) (the lasso with D = I)."""
    b, _ = case(91, 2, 1, 1, (32, 32), (1, 1))
    d = np.ones((1, 1, 1, 1), np.float32)
    beta = 2.0
    z = N(lib.code(T(b), T(d), beta, 1.0, 200)[0])
    x = b.astype(np.float64)
    soft = np.sign(x) * np.maximum(np.abs(x) - beta, 0.0)
    assert np.count_nonzero(soft) > 0.1 * soft.size
    assert np.abs(z - soft).max() <= 1e-4 * max(1.0, np.abs(soft).max())


@pytest.mark.parametrize("grid,k,fs,n,amp,beta", [
    ((64, 64), 1, (11, 11), 2, 10.0, 1.0),     # one filter
    ((16, 16), 3, (16, 16), 2, 10.0, 1.0),     # support as large as the grid (largest pruned support)
    ((8, 32), 3, (5, 11), 2, 10.0, 1.0),       # H = 8: one pass-A workgroup holds every canonical row
    ((16, 64), 2, (1, 1), 3, 0.1, 0.01),       # 1 x 1 support (scaled, see below)
    ((128, 128), 4, (7, 11), 1, 10.0, 1.0),    # N = 1, non-square support
])
@pytest.mark.parametrize("form", ["span", "direct"])
def test_learn_degenerate_shapes(lib, grid, k, fs, n, amp, beta, form):
    """With a 1 x 1 support the learning operator is I plus a rank-K term
    whose eigenvalues are about 1 + |z_k|^2 / (2 mu_k): at the usual
    amplitude (codes ~10 over 3000 pixels) its condition number is ~4e4, and
    float32 CG cannot follow the FP64 solve to 1e-4.  That case runs on
    images and beta scaled by 0.01 (codes scaled by 0.01; condition ~5), the
    same problem up to scale."""
    b, d0 = case(101 + k, n, 1, k, grid, fs, amp=amp)
    z = oracle.code(b, d0, beta, 5.0, 10)["z"].astype(np.float32)
    assert np.count_nonzero(z) > 0
    mu0 = np.linspace(0.8, 1.5, k).astype(np.float32)
    d_ref, mu_ref, g_ref = oracle.learn(b, z, fs, mu0, None, 3, 6)
    d, mu, gamma = lib.learn(T(b), T(z), fs, T(mu0), None, 3, 6, form=form)
    assert np.abs(N(d) - d_ref).max() <= 1e-4 * max(1.0, float(np.abs(d_ref).max()))
    np.testing.assert_allclose(N(mu), mu_ref, rtol=1e-4)
    assert np.abs(N(gamma) - g_ref).max() <= 1e-4 * max(1.0, float(np.abs(g_ref).max()))


def test_check_finite(lib):
    """Non-finite detection (csc_check_finite through the binding): finite
    data passes; a NaN, +inf or -inf anywhere (also the last element of a
    tensor larger than one pass of the grid) raises CSC_ENONFINITE; an empty
    tensor passes."""
    import torch
    x = torch.randn(3_000_001, device="cuda")
    lib.check_finite(x, torch.zeros(0, device="cuda"))
    for bad, at in ((float("nan"), 17), (float("inf"), -1), (float("-inf"), 1_500_000)):
        y = x.clone()
        y[at] = bad
        with pytest.raises(lib.DualCSCError) as e:
            lib.check_finite(x, y)
        assert e.value.code == lib.ENONFINITE
    lib.check_finite(x)
