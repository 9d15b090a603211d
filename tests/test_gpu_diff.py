"""Differentiable unrolled coding on the GPU: forward parity with the FP64
oracle, loss gradients, and gradients with respect to the filters and beta
against the oracle's reverse pass (itself pinned by FP64 finite differences
in test_oracle.py).  Gradient tolerance: 1e-3 of max |grad| (float32
forward and adjoint through 30 iterations)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3


def T(x, grad=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    return t.requires_grad_(grad)


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_unrolled_forward_matches_oracle(lib):
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg, n=2)
    z = lib.unrolled_code(T(b), T(d), cfg.beta, cfg.rho, 12, 5)
    ref = oracle.code(b, d, cfg.beta, cfg.rho, 12)["z"]
    assert np.count_nonzero(ref) > 0
    assert np.abs(N(z) - ref).max() <= 1e-4


def test_unrolled_forward_is_the_coding_iteration(lib):
    """The unrolled forward runs csc_code's iteration: equal z bit for bit,
    with checkpoints recorded or not, on the split-path grid too."""
    for grid, n in (((64, 64), 2), ((256, 256), 1)):
        rng = np.random.default_rng(11)
        b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, grid))[None] * 30 for _ in range(n)])
        d = synth.unit_filters(6, 1, (11, 11), 3)
        z_code = N(lib.code(T(b), T(d), 1.0, 10.0, 9)[0])
        for every in (1, 4, 9):
            z = N(lib.unrolled_code(T(b), T(d), 1.0, 10.0, 9, every))
            assert np.array_equal(z, z_code), (grid, every)


@pytest.mark.parametrize("split", [False, True])
def test_unrolled_records_hold_the_states(lib, split):
    """Records 0, 1, 2 of iters = 9, every = 4 hold (z, theta) after 0, 4
    and 8 iterations (csc_code's, bit for bit), at the record stride the
    library reports, and nothing is written past the last record; on a
    single-tile grid and on a 128 x 256 grid (split path, where record
    iterations write their codes straight into the record)."""
    import ctypes
    import torch
    cfg = synth.CONFIGS["small"]
    if split:
        rng = np.random.default_rng(12)
        b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, (128, 256)))[None] * 10 for _ in range(2)])
        b = b.astype(np.float32)
        d = synth.unit_filters(cfg.k, 1, (11, 11), 5)
    else:
        b, d = synth.make_inputs(cfg, n=2)
    bt, dt = T(b), T(d)
    shape = lib._shape_of(bt, dt)
    L = lib.load()
    rec = L.csc_unrolled_record_floats(ctypes.byref(shape))
    nz = cfg.k * 2 * b.shape[2] * b.shape[3]
    assert rec == 2 * nz + 6 * 2 * b.shape[2] * b.shape[3]
    rho = torch.full((2,), cfg.rho, dtype=torch.float32, device="cuda")
    z = torch.empty((2, cfg.k) + b.shape[2:], dtype=torch.float32, device="cuda")
    ckpt = torch.full((3 * rec + 1024,), 7.0, dtype=torch.float32, device="cuda")
    ws, nbytes = lib._diff_ws(shape, 4, bt.device)
    rc = L.csc_code_unrolled(ctypes.byref(shape), lib._ptr(bt), lib._ptr(dt), cfg.beta, lib._ptr(rho), 9, 4,
                             lib._ptr(z), lib._ptr(ckpt), ws, nbytes, lib._stream())
    assert rc == 0
    torch.cuda.synchronize()
    c = ckpt.cpu().numpy()
    assert np.all(c[3 * rec:] == 7.0)
    assert np.all(c[:2 * nz] == 0.0)
    for r, it in ((1, 4), (2, 8)):
        zr, thr = lib.code(bt, dt, cfg.beta, cfg.rho, it, want_theta=True)[:2]
        assert np.array_equal(c[r * rec:r * rec + nz], zr.cpu().numpy().ravel()), r
        assert np.array_equal(c[r * rec + nz:r * rec + 2 * nz], thr.cpu().numpy().ravel()), r


def test_loss_grad_matches_oracle(lib):
    import torch
    b, d = synth.make_inputs(synth.CONFIGS["small"], n=2)
    z0 = oracle.code(b, d, 1.0, 10.0, 8)["z"].astype(np.float32)
    dt, zt = T(d, True), T(z0, True)
    beta = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    L = lib.csc_loss(T(b), dt, zt, beta)
    L.backward()
    f, dz, dd, db = oracle.objective_grad(b, d, z0, 0.7)
    assert abs(L.item() - f) <= 1e-5 * abs(f)
    assert np.abs(N(zt.grad) - dz).max() <= 1e-4 * max(1.0, np.abs(dz).max())
    assert np.abs(N(dt.grad) - dd).max() <= 1e-5 * np.abs(dd).max()
    assert abs(beta.grad.item() - db) <= 1e-5 * db


def check_grads(gd, gb, gdr, gbr):
    """Filter and beta gradients each within GRAD_RTOL of their own size."""
    ed = np.abs(gd - gdr).max() / np.abs(gdr).max()
    eb = abs(gb - gbr) / abs(gbr)
    print("gradient errors: filters %.2e of max|dL/dd|, beta %.2e relative" % (ed, eb))
    assert ed <= GRAD_RTOL, ed
    assert eb <= GRAD_RTOL, eb


def unrolled_grad(lib, b, d, beta, rho, iters, every):
    import torch
    dt = T(d, True)
    bt = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    z = lib.unrolled_code(T(b), dt, bt, rho, iters, every)
    L = lib.csc_loss(T(b), dt, z, bt)
    L.backward()
    return L.item(), N(dt.grad), bt.grad.item()


def test_gradient_fd_instance_vs_oracle(lib):
    """2 x 32x32 images, K = 4 filters 11x11, 30 iterations, checkpoint every 5."""
    cfg = synth.CONFIGS["unrolled_fd"]
    b, d = synth.make_inputs(cfg)
    L, gd, gb = unrolled_grad(lib, b, d, cfg.beta, cfg.rho, cfg.t_in, 5)
    Lr, gdr, gbr = oracle.code_loss_grad(b, d, cfg.beta, cfg.rho, cfg.t_in)
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    check_grads(gd, gb, gdr, gbr)


def test_gradient_larger_instance_vs_oracle(lib):
    rng = np.random.default_rng(4)
    b = np.stack([synth.contrast_normalize(synth.one_over_f(rng, (64, 64)))[None] * 30 for _ in range(2)])
    d = synth.unit_filters(8, 1, (11, 11), 77)
    L, gd, gb = unrolled_grad(lib, b, d, 1.0, 10.0, 10, 4)
    Lr, gdr, gbr = oracle.code_loss_grad(b, d, 1.0, 10.0, 10)
    check_grads(gd, gb, gdr, gbr)


def test_checkpoint_interval_does_not_change_gradient(lib):
    cfg = synth.CONFIGS["unrolled_fd"]
    b, d = synth.make_inputs(cfg)
    ref = unrolled_grad(lib, b, d, cfg.beta, cfg.rho, 12, 1)
    for every in (3, 5, 12):
        got = unrolled_grad(lib, b, d, cfg.beta, cfg.rho, 12, every)
        assert np.array_equal(got[1], ref[1]) and got[2] == ref[2], every


@pytest.mark.parametrize("grid,fs", [((128, 256), (11, 11)), ((4, 16, 16), (3, 5, 5))])
def test_gradient_axis_path_grids(lib, grid, fs):
    """Grids transformed axis by axis (beyond one LDS tile, and a 3-D volume),
    where the adjoint folds its elementwise steps into the transform passes:
    gradient against the oracle's reverse pass, bit-identical for checkpoint
    intervals 2 and 5."""
    rng = np.random.default_rng(8 if len(grid) == 2 else 9)
    b = (synth.contrast_normalize(synth.one_over_f(rng, grid)) * 30)[None, None]
    d = synth.unit_filters(4 if len(grid) == 2 else 3, 1, fs, 78 if len(grid) == 2 else 79)
    ref = unrolled_grad(lib, b, d, 1.0, 10.0, 8, 2)
    got = unrolled_grad(lib, b, d, 1.0, 10.0, 8, 5)
    assert np.array_equal(got[1], ref[1]) and got[2] == ref[2]
    Lr, gdr, gbr = oracle.code_loss_grad(b, d, 1.0, 10.0, 8)
    assert abs(ref[0] - Lr) <= 1e-5 * abs(Lr)
    check_grads(ref[1], ref[2], gdr, gbr)


def test_zero_iterations(lib):
    import torch
    cfg = synth.CONFIGS["unrolled_fd"]
    b, d = synth.make_inputs(cfg)
    dt = T(d, True)
    z = lib.unrolled_code(T(b), dt, 1.0, 10.0, 0, 5)
    assert torch.count_nonzero(z).item() == 0
    L = lib.csc_loss(T(b), dt, z, 1.0)
    L.backward()
    assert torch.count_nonzero(dt.grad).item() == 0
