"""GPU parity of the nuclear-norm regulariser (Sec. 5: low-rank code maps;
CSC_NUCLEAR) against the FP64 oracle's code(reg="nuclear"): codes within
1e-4 max-abs after a fixed iteration count, objectives within 1e-5
relative.  Inputs: the 4 x 64^2, K = 16 workload with beta = 10 (code maps
of rank 3..8 of 64 after 20 iterations), rectangular grids in both
orientations, odd K (a half-empty filter pair), J = 3, adaptive rho."""
import numpy as np
import pytest

import oracle
import synth
from tolerances import CODE_TOL, OBJ_RTOL

pytestmark = pytest.mark.gpu

BETA_NUC = 10.0


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def ranks(z):
    s = np.linalg.svd(z, compute_uv=False)
    return (s > 1e-6 * max(1.0, s.max())).sum(-1)


def test_nuclear_small_config(lib):
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg)
    print("nuclear: 4 x 64^2, K=16, beta 10", flush=True)
    ref = oracle.code(b, d, BETA_NUC, cfg.rho, cfg.t_in, reg="nuclear")
    z, th, resid, _ = lib.code(T(b), T(d), BETA_NUC, cfg.rho, cfg.t_in, want_theta=True, want_resid=True,
                               reg="nuclear")
    r = ranks(ref["z"])
    assert 0 < r.min() and r.max() < 16, r
    err = np.abs(N(z) - ref["z"]).max()
    eth = np.abs(N(th) - ref["theta"]).max()
    print("codes %.2e, theta %.2e, ranks %d..%d" % (err, eth, r.min(), r.max()))
    assert err <= CODE_TOL, err
    assert eth <= CODE_TOL, eth
    np.testing.assert_allclose(N(resid)[:, :, :2], ref["resid"], rtol=1e-3, atol=1e-6)
    obj = N(lib.objective(T(b), T(d), z, BETA_NUC, reg="nuclear"))
    per, tot = oracle.objective(b, d, N(z), BETA_NUC, reg="nuclear")
    assert abs(obj[-1] - tot) <= OBJ_RTOL * abs(tot), (obj[-1], tot)
    np.testing.assert_allclose(obj[:-1], per, rtol=OBJ_RTOL)


@pytest.mark.parametrize("grid,k,j,beta", [((32, 64), 5, 1, 6.0), ((64, 32), 4, 1, 6.0), ((32, 32), 6, 3, 6.0),
                                           ((16, 8), 3, 1, 2.0), ((128, 128), 9, 1, 12.0)])
def test_nuclear_shapes(lib, grid, k, j, beta):
    rng = np.random.default_rng(31)
    b = np.stack([np.stack([synth.contrast_normalize(synth.one_over_f(rng, grid)) * 10 for _ in range(j)])
                  for _ in range(2)]).astype(np.float32)
    d = synth.unit_filters(k, j, (5, 5), 32)
    print("nuclear shape", grid, k, j, flush=True)
    ref = oracle.code(b, d, beta, 10.0, 12, reg="nuclear")
    z, _, _, _ = lib.code(T(b), T(d), beta, 10.0, 12, reg="nuclear")
    r = ranks(ref["z"])
    assert r.max() > 0 and r.min() < min(grid), r
    err = np.abs(N(z) - ref["z"]).max()
    assert err <= CODE_TOL, err


def test_nuclear_warm_start_adaptive(lib):
    """Two calls chained through z and theta with adaptive rho: the GPU's rho
    schedule replayed in the oracle."""
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg, n=2)
    z, th, res1, rho = lib.code(T(b), T(d), BETA_NUC, cfg.rho, 6, want_theta=True, want_resid=True, adaptive=True,
                                reg="nuclear")
    z, th, res2, rho = lib.code(T(b), T(d), BETA_NUC, rho, 6, z=z, theta=th, want_resid=True, adaptive=True,
                                reg="nuclear")
    sched = np.concatenate([N(res1)[:, :, 2], N(res2)[:, :, 2], N(rho)[None]])
    ref = oracle.code(b, d, BETA_NUC, cfg.rho, 12, rho_schedule=sched, reg="nuclear")
    err = np.abs(N(z) - ref["z"]).max()
    assert err <= CODE_TOL, err
    assert np.abs(N(th) - ref["theta"]).max() <= CODE_TOL


def test_nuclear_rejects_unsupported(lib):
    import torch
    b = torch.zeros((1, 1, 256, 256), device="cuda")
    d = torch.zeros((2, 1, 5, 5), device="cuda")
    with pytest.raises(lib.DualCSCError):
        lib.code(b, d, 1.0, 1.0, 2, reg="nuclear")
