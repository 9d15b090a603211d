"""hipGraph capture/replay of csc_code and csc_learn: every replay equals the
eager call bitwise, with unrelated eager work and synchronisations between
the replays."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def test_learn_graph_replays_equal_eager(lib):
    import torch
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg)
    bt, dt = T(b), T(d0)
    z, _, _, _ = lib.code(bt, dt, cfg.beta, cfg.rho, 10)
    mu0 = torch.ones(cfg.k, device="cuda")
    d_e, mu_e, g_e = lib.learn(bt, z, cfg.fsupp, mu0.clone(), None, 3, 4)
    d_out = torch.empty_like(d_e)
    mu = torch.empty_like(mu0)
    gamma = torch.empty_like(bt)
    for rep in range(3):
        mu.copy_(mu0)
        gamma.zero_()
        lib.learn(bt, z, cfg.fsupp, mu, gamma, 3, 4, out=d_out, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(d_out, d_e) and torch.equal(mu, mu_e) and torch.equal(gamma, g_e), rep
        lib.code(bt, dt, cfg.beta, cfg.rho, 2)
        torch.cuda.synchronize()


def test_code_graph_replays_equal_eager(lib):
    import torch
    cfg = synth.CONFIGS["small"]
    b, d0 = synth.make_inputs(cfg)
    bt, dt = T(b), T(d0)
    z_e, _, _, _ = lib.code(bt, dt, cfg.beta, cfg.rho, 7)
    z = torch.empty_like(z_e)
    th = torch.empty_like(z_e)
    rho = torch.empty(cfg.n, device="cuda")
    for rep in range(3):
        z.zero_()
        th.zero_()
        rho.fill_(cfg.rho)
        lib.code(bt, dt, cfg.beta, rho, 7, z=z, theta=th, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(z, z_e), rep
        lib.learn(bt, z_e, cfg.fsupp, None, None, 1, 2)
        torch.cuda.synchronize()


def test_trace_sampling_counts(lib):
    """csc_trace_enable(n) brackets the 1st, (n+1)-th, ... launch of a class:
    7 coding iterations give 7 records with n = 1 and 3 with n = 3."""
    import torch
    rng = np.random.default_rng(3)
    b = torch.from_numpy(rng.standard_normal((2, 1, 64, 64)).astype(np.float32)).cuda()
    d = torch.from_numpy(rng.standard_normal((4, 1, 11, 11)).astype(np.float32)).cuda()
    for every, want in ((1, 7), (3, 3)):
        lib.trace_enable(True, every=every)
        lib.code(b, d, 1.0, 5.0, 7)
        torch.cuda.synchronize()
        lib.trace_enable(False)
        ms, cnt = lib.trace_read(lib.TRACE_CODE_MAPS)
        assert cnt == want and ms > 0.0
