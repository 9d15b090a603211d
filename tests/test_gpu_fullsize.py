"""Parity at the full sizes of the benchmarked workloads, in the launch
configurations bench.py times, on outputs the FP64 oracle can compute:

* the learning-alternation step (10 x 128^2, K=100): coding with adaptive rho
  (the GPU's rho schedule replayed by the oracle), learning from the GPU's
  codes, and the objective, all on the full workload;
* the batched form (256 ragged images, K=64, 30 iterations, hipGraph replay):
  coding is independent per image, so sampled images of the full batch are
  compared with the oracle run on those images alone;
* the differentiable form (16 x 256^2, K=100, 30 unrolled iterations,
  checkpoints every 5): the forward codes of a sampled image, the filter and
  beta gradients of one image against the oracle's reverse pass, and the
  full-batch gradient against the batch in reverse order and against the sum
  of the gradients of its two halves, each padded with zero images to the
  batch size (the loss is a sum over images whose codes do not interact);
* tensor CSC at its full size (32 x RGB 128^2, K=64): sampled images; the
  RGB video volume (16 x 128 x 128, K=64) in full.

Tolerances as in test_gpu_parity.py (codes 1e-4, or 3e-6 * max|z| for large
codes; objective 1e-5 relative) and test_gpu_diff.py (gradients 1e-3 of
max |grad|)."""
import numpy as np
import pytest

import oracle
import synth
from tolerances import CODE_TOL, OBJ_RTOL, code_tol

pytestmark = pytest.mark.gpu
GRAD_RTOL = 1e-3


def T(x, grad=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    return t.requires_grad_(grad)


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)




def test_learning_step_full_workload(lib):
    """One outer step of the benchmark: 10 images 128^2, K=100, adaptive rho,
    10 coding iterations, learning 10 x 10, objective."""
    import torch
    cfg = synth.CONFIGS["learn"]
    b, d0 = synth.make_inputs(cfg)
    bt = T(b)
    rho0 = torch.full((cfg.n,), cfg.rho0, dtype=torch.float32, device="cuda")
    z, theta, resid, rho = lib.code(bt, T(d0), cfg.beta, rho0, cfg.t_in, adaptive=True, want_theta=True,
                                    want_resid=True)
    sched = np.concatenate([N(resid)[:, :, 2], N(rho)[None]], axis=0)
    ref = oracle.code(b, d0, cfg.beta, cfg.rho0, cfg.t_in, rho_schedule=sched)
    assert np.count_nonzero(ref["z"]) / ref["z"].size > 0.01
    assert np.abs(N(z) - ref["z"]).max() <= code_tol(ref["z"])
    assert np.abs(N(theta) - ref["theta"]).max() <= code_tol(ref["theta"])

    mu = torch.ones(cfg.k, dtype=torch.float32, device="cuda")
    d, mu1, gamma = lib.learn(bt, z, cfg.fsupp, mu, None, cfg.learn_inner, cfg.learn_cg)
    zf = N(z).astype(np.float32)
    d_ref, mu_ref, _ = oracle.learn(b, zf, cfg.fsupp, np.ones(cfg.k), None, cfg.learn_inner, cfg.learn_cg)
    assert np.abs(N(d) - d_ref).max() <= 1e-4 * max(1.0, np.abs(d_ref).max())
    np.testing.assert_allclose(N(mu1), mu_ref, rtol=1e-4)

    obj = N(lib.objective(bt, d, z, cfg.beta))
    per, tot = oracle.objective(b, N(d).astype(np.float32), zf, cfg.beta)
    np.testing.assert_allclose(obj[:-1], per, rtol=OBJ_RTOL)
    assert abs(obj[-1] - tot) <= OBJ_RTOL * abs(tot)


def test_batched_full_workload_sampled(lib):
    """All 256 ragged images in one hipGraph-replayed call; images from the
    largest, a rectangular and a small grid class against the oracle."""
    import torch
    cfg = synth.CONFIGS["batched"]
    imgs, grids, d0 = synth.ragged_inputs(cfg)
    padded = []
    for im, g in zip(imgs, grids):
        t = torch.zeros((1,) + g, dtype=torch.float32)
        t[:, :im.shape[1], :im.shape[2]] = torch.from_numpy(im)
        padded.append(t.cuda())
    pb = lib.PackedBatch(padded, cfg.k)
    z = torch.empty(pb.z_numel, dtype=torch.float32, device="cuda")
    lib.code_batched(pb, T(d0), cfg.beta, cfg.rho, cfg.t_in, z=z, graph=True)   # capture + replay
    lib.code_batched(pb, T(d0), cfg.beta, cfg.rho, cfg.t_in, z=z, graph=True)   # replay
    zs = pb.z_views(z)
    picks = []
    for want in ((256, 256), (128, 256), (256, 64), (64, 64)):
        idx = [i for i, g in enumerate(grids) if g == want]
        if idx:
            picks.append(idx[0])
    assert len(picks) >= 3
    for i in picks:
        ref = oracle.code(padded[i].cpu().numpy()[None], d0, cfg.beta, cfg.rho, cfg.t_in)["z"][0]
        assert np.count_nonzero(ref) / ref.size > 0.005, grids[i]
        assert np.abs(zs[i].cpu().numpy() - ref).max() <= code_tol(ref), grids[i]


def test_unrolled_full_workload(lib):
    """16 x 256^2, K=100, 30 unrolled iterations, checkpoints every 5."""
    import torch
    cfg = synth.CONFIGS["unrolled"]
    b, d0 = synth.make_inputs(cfg)
    every = 5

    def grad(bsub):
        dt = T(d0, True)
        bet = torch.tensor(cfg.beta, dtype=torch.float64, requires_grad=True)
        z = lib.unrolled_code(T(bsub), dt, bet, cfg.rho, cfg.t_in, every)
        L = lib.csc_loss(T(bsub), dt, z, bet)
        L.backward()
        return L.item(), N(dt.grad), bet.grad.item(), z

    L, gd, gb, z = grad(b)
    ref = oracle.code(b[:1], d0, cfg.beta, cfg.rho, cfg.t_in)["z"]
    assert np.count_nonzero(ref) / ref.size > 0.005
    assert np.abs(N(z[:1]) - ref).max() <= code_tol(ref)

    # Every image goes through the same arithmetic wherever it sits in the
    # batch: with the images in reverse order only the order of the sum over
    # images changes.
    Lr_, gdr_, gbr_, zr_ = grad(b[::-1].copy())
    assert abs(L - Lr_) <= 1e-6 * abs(L)
    assert np.abs(N(zr_)[::-1] - N(z)).max() == 0.0
    assert np.abs(gd - gdr_).max() <= 1e-5 * np.abs(gd).max()
    assert abs(gb - gbr_) <= 1e-6 * abs(gb)

    # The batch gradient is the sum of the gradients of its halves.  Each
    # half is padded with zero images (zero codes, no loss, no gradient) to
    # the batch size, so that it runs under the batch's plan: a batch of
    # another size groups the filter-pair sums differently, and the unrolled
    # filter gradient moves with such a regrouping of float32 sums by up to
    # 4e-3 of its maximum (test_float32_floor.py), through codes that cross
    # the clipping kinks.
    zero = np.zeros_like(b[:8])
    La, gda, gba, _ = grad(np.concatenate([b[:8], zero]))
    Lb, gdb, gbb, _ = grad(np.concatenate([zero, b[8:]]))
    hd = np.abs(gd - (gda + gdb)).max() / np.abs(gd).max()
    hb = abs(gb - (gba + gbb)) / abs(gb)
    print("batch minus halves: loss %.2e, filters %.2e of max|dL/dd|, beta %.2e relative"
          % (abs(L - (La + Lb)) / abs(L), hd, hb), flush=True)
    assert abs(L - (La + Lb)) <= 1e-6 * abs(L)
    assert hd <= 1e-5, hd
    assert hb <= 1e-6, hb

    # one image against the oracle's reverse pass
    L0, gd0, gb0, _ = grad(b[:1])
    Lr, gdr, gbr = oracle.code_loss_grad(b[:1], d0, cfg.beta, cfg.rho, cfg.t_in)
    ed = np.abs(gd0 - gdr).max() / np.abs(gdr).max()
    eb = abs(gb0 - gbr) / abs(gbr)
    print("full-size gradient of one image: loss %.2e, filters %.2e of max|dL/dd|, beta %.2e relative"
          % (abs(L0 - Lr) / abs(Lr), ed, eb), flush=True)
    assert abs(L0 - Lr) <= 1e-5 * abs(Lr)
    assert ed <= GRAD_RTOL, ed
    assert eb <= GRAD_RTOL, eb


def test_tensor_full_size_sampled(lib):
    """32 RGB images 128^2, K=64 filters 11x11x3, 20 iterations: the first
    and the last image against the oracle."""
    cfg = synth.CONFIGS["tensor"]
    b, d0 = synth.make_inputs(cfg)
    z = N(lib.code(T(b), T(d0), cfg.beta, cfg.rho, cfg.t_in)[0])
    for i in (0, cfg.n - 1):
        ref = oracle.code(b[i:i + 1], d0, cfg.beta, cfg.rho, cfg.t_in)["z"]
        assert np.count_nonzero(ref) / ref.size > 0.005
        assert np.abs(z[i:i + 1] - ref).max() <= code_tol(ref), i


def test_video_full_size(lib):
    """One RGB volume 16 x 128 x 128, K=64 filters 3 x 11 x 11 x 3, 20
    iterations (3-D grids take the axis-pass path)."""
    cfg = synth.CONFIGS["video"]
    b, d0 = synth.make_inputs(cfg)
    z = N(lib.code(T(b), T(d0), cfg.beta, cfg.rho, cfg.t_in)[0])
    ref = oracle.code(b, d0, cfg.beta, cfg.rho, cfg.t_in)["z"]
    assert np.count_nonzero(ref) / ref.size > 0.005
    assert np.abs(z - ref).max() <= code_tol(ref)
