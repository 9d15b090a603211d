"""The float32 floor behind the GPU tolerances that exceed the contract.

The oracle's algorithm is run in float32 (tests/f32_emulation.py) and
compared with the oracle in float64 on the same inputs.  Each bound in
tests/tolerances.py that is looser than the contract must lie between the
largest distance measured here and twice that, so that it is neither below
what float32 can reach nor far above it.
"""
import numpy as np
import pytest

import oracle
import synth
import tolerances as tol
import f32_emulation as f32


def _perturbed(b, seed):
    """The images with every value moved by one float32 ulp up or down."""
    if seed == 0:
        return np.asarray(b, np.float32)
    rng = np.random.default_rng(seed)
    return (np.asarray(b, np.float32) * (1 + rng.choice([-1, 1], b.shape) * 2.0 ** -24)).astype(np.float32)


def _within_floor(bound, floor):
    return floor <= bound <= 2.0 * floor


def test_chained_alternation_floor():
    """Alg. 1, two outer steps on the 4 x 64^2, K = 16 workload (beta 1, rho
    10, 20 coding iterations, learning 10 x 10): four float32 runs (the
    images as given and moved by one ulp with three seeds) against the
    float64 oracle on the images as given."""
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg)
    ref = oracle.learn_dictionary(b, d0, cfg.beta, cfg.rho, cfg.t_in, cfg.t_out, cfg.learn_inner, cfg.learn_cg)
    dz = dd = dobj = dmu = 0.0
    for seed in range(4):
        d, z, mu, states = f32.learn_dictionary(_perturbed(b, seed), d0, cfg.beta, cfg.rho, cfg.t_in, cfg.t_out,
                                                cfg.learn_inner, cfg.learn_cg)
        dz = max(dz, float(np.abs(z - ref["z"]).max()))
        dd = max(dd, float(np.abs(d - ref["d"]).max()))
        dmu = max(dmu, float(np.abs(mu / ref["mu"] - 1).max()))
        for (zs, ds), f_ref in zip(states, ref["objectives"]):
            dobj = max(dobj, abs(oracle.objective(b, ds, zs, cfg.beta)[1] - f_ref) / abs(f_ref))
    print("float32 floor of the chained run: codes %.3e, filters %.3e, objective %.3e, mu %.3e"
          % (dz, dd, dobj, dmu))
    # the contract itself is below the floor for the codes
    assert dz > tol.CODE_TOL
    assert _within_floor(tol.CHAIN_CODE_TOL, dz), (tol.CHAIN_CODE_TOL, dz)
    assert _within_floor(tol.CHAIN_FILTER_TOL, dd), (tol.CHAIN_FILTER_TOL, dd)
    assert _within_floor(tol.CHAIN_OBJ_RTOL, dobj), (tol.CHAIN_OBJ_RTOL, dobj)
    assert _within_floor(tol.CHAIN_MU_RTOL, dmu), (tol.CHAIN_MU_RTOL, dmu)


def test_large_amplitude_coding_floor():
    """One coding call (beta 1, rho 10, 30 iterations, K = 64 11 x 11) on
    ragged images times 30: float32 against float64, relative to max|z|."""
    cfg = synth.CONFIGS["batched"]
    imgs, grids, d = synth.ragged_inputs(cfg, n=3)
    worst = 0.0
    for im, g in zip(imgs, grids):
        x = np.zeros((1, 1) + g, np.float32)
        x[0, :, :im.shape[1], :im.shape[2]] = im
        ref = oracle.code(x, d, cfg.beta, cfg.rho, cfg.t_in)["z"]
        z, _ = f32.code(x, d, cfg.beta, cfg.rho, cfg.t_in)
        ratio = float(np.abs(z - ref).max() / np.abs(ref).max())
        print("grid %s: max|z| %.1f, float32 floor %.2e of max|z|" % (g, np.abs(ref).max(), ratio))
        assert np.abs(ref).max() * ratio > tol.CODE_TOL  # 1e-4 absolute is below the floor here
        worst = max(worst, ratio)
    assert _within_floor(tol.LARGE_CODE_RTOL, worst), (tol.LARGE_CODE_RTOL, worst)


def test_emulation_is_the_oracle_in_float32():
    """The emulation follows the oracle's steps: on a small case its result
    is the oracle's to float32 accuracy (a wrong sign or dropped term would
    leave an O(1) difference)."""
    rng = np.random.default_rng(3)
    b = (rng.standard_normal((2, 1, 16, 16)) * 3).astype(np.float32)
    d = synth.unit_filters(3, 1, (5, 5), 4)
    ref = oracle.code(b, d, 0.5, 2.0, 15)
    z, th = f32.code(b, d, 0.5, 2.0, 15)
    assert np.abs(z - ref["z"]).max() <= 1e-4 * max(1.0, np.abs(ref["z"]).max())
    assert np.abs(th - ref["theta"]).max() <= 1e-4
    d_ref, mu_ref, g_ref = oracle.learn(b, ref["z"].astype(np.float32), (5, 5), np.ones(3), None, 3, 6)
    d32, mu32, g32 = f32.learn(b, ref["z"].astype(np.float32), (5, 5), np.ones(3), None, 3, 6)
    assert np.abs(d32 - d_ref).max() <= 1e-4
    np.testing.assert_allclose(mu32, mu_ref, rtol=1e-4)


@pytest.mark.parametrize("grid,k", [((256, 256), 4), ((128, 256), 6)])
def test_unrolled_gradient_floor(grid, k):
    """The filter gradient of the unrolled solve (2 images, 10 iterations,
    beta 1, rho 10, images times 30) in float32 against float64: on grids
    transformed axis by axis the float32 floor is above 1e-4 of max|dL/dd|
    (so that gradients are compared at 1e-3 of their maximum, not 1e-4),
    while the beta gradient stays near 1e-6."""
    rng = np.random.default_rng(21)
    b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, grid))[None] * 30 for _ in range(2)])
    b = b.astype(np.float32)
    d = synth.unit_filters(k, 1, (11, 11), 5)
    _, gdr, gbr = oracle.code_loss_grad(b, d, 1.0, 10.0, 10)
    _, gd, gb = f32.code_loss_grad(b, d, 1.0, 10.0, 10)
    ed = float(np.abs(gd - gdr).max() / np.abs(gdr).max())
    eb = abs(gb - gbr) / abs(gbr)
    print("grid %s K=%d: float32 floor of the filter gradient %.2e of max, beta %.2e" % (grid, k, ed, eb))
    assert 5e-5 < ed < 1e-3, ed
    assert eb < 1e-5, eb


def test_unrolled_gradient_regrouping():
    """How far a regrouping of float32 sums alone moves the unrolled filter
    gradient (2 images 128^2, K = 32, 30 iterations, beta 1, rho 10, images
    times 30): the float32 solve with its filters in three shuffled orders
    against the float32 solve in the given order.  A different grouping
    moves some codes across the clipping kinks, and the gradient by more
    than 1e-3 of its maximum; gradients of batches of different sizes (which
    the GPU groups differently) are therefore not compared with each other."""
    rng = np.random.default_rng(21)
    b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, (128, 128)))[None] * 30 for _ in range(2)])
    b = b.astype(np.float32)
    d = synth.unit_filters(32, 1, (11, 11), 5)
    _, gd, gb = f32.code_loss_grad(b, d, 1.0, 10.0, 30)
    worst = 0.0
    for seed in range(3):
        perm = np.random.default_rng(seed).permutation(d.shape[0])
        _, gdp, gbp = f32.code_loss_grad(b, d[perm], 1.0, 10.0, 30)
        gdp = gdp[np.argsort(perm)]
        worst = max(worst, float(np.abs(gd - gdp).max() / np.abs(gd).max()))
        assert abs(gb - gbp) < 1e-4 * abs(gb)
    print("regrouped float32 sums move the filter gradient by %.2e of its max" % worst)
    assert 1e-3 < worst < 1e-2, worst
