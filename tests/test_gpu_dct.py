"""GPU parity of the DCT-domain variant (symmetric boundaries, csc_code_dct)
against the FP64 oracle of oracle/dct.py: codes within 1e-4 max-abs after a
fixed iteration count, objectives within 1e-5 relative.  Inputs: 1/f
contrast-normalised images times 10, whole-sample symmetric 11 x 11 filters
(6 x 6 quadrants, unit norm), beta = 1, rho = 10, on 64^2 and 128^2 grids,
rectangular grids both ways, odd K, J = 3, warm starts and adaptive rho."""
import numpy as np
import pytest

import synth
from oracle import dct
from tolerances import CODE_TOL, OBJ_RTOL, code_tol

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def images(n, j, grid, seed, amp=10.0):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([synth.contrast_normalize(synth.one_over_f(rng, grid)) * amp for _ in range(j)])
                     for _ in range(n)]).astype(np.float32)


@pytest.mark.parametrize("grid,n,k,j,m", [((64, 64), 4, 16, 1, (6, 6)), ((128, 128), 2, 20, 1, (6, 6)),
                                          ((32, 64), 2, 5, 1, (4, 3)), ((64, 16), 2, 4, 1, (3, 5)),
                                          ((32, 32), 2, 6, 3, (6, 6)), ((8, 8), 3, 3, 1, (2, 2))])
def test_dct_code_matches_oracle(lib, grid, n, k, j, m):
    b = images(n, j, grid, 40 + grid[0] + k)
    q = synth.symmetric_quadrants(k, j, m, 41)
    print("dct coding", grid, n, k, j, m, flush=True)
    ref = dct.code(b, q, 1.0, 10.0, 20)
    z, th, resid, _ = lib.code_dct(T(b), T(q), 1.0, 10.0, 20, want_theta=True, want_resid=True)
    dens = np.count_nonzero(ref["z"]) / ref["z"].size
    err = np.abs(N(z) - ref["z"]).max()
    print("density %.3f, codes %.2e, theta %.2e" % (dens, err, np.abs(N(th) - ref["theta"]).max()))
    assert dens > 0.005, dens
    assert err <= code_tol(ref["z"]), err
    assert np.abs(N(th) - ref["theta"]).max() <= CODE_TOL
    np.testing.assert_allclose(N(resid)[:, :, :2], ref["resid"], rtol=1e-3, atol=1e-6)
    obj = N(lib.objective_dct(T(b), T(q), z, 1.0))
    per, tot = dct.objective(b, q, N(z), 1.0)
    assert abs(obj[-1] - tot) <= OBJ_RTOL * abs(tot), (obj[-1], tot)
    np.testing.assert_allclose(obj[:-1], per, rtol=OBJ_RTOL)


def test_dct_warm_start_and_adaptive_rho(lib):
    """Two chained calls (z and theta carried) with adaptive rho: the GPU's
    schedule replayed by the oracle."""
    b = images(3, 1, (64, 64), 50)
    q = synth.symmetric_quadrants(8, 1, (6, 6), 51)
    z, th, r1, rho = lib.code_dct(T(b), T(q), 1.0, 10.0, 7, want_theta=True, want_resid=True, adaptive=True)
    z, th, r2, rho = lib.code_dct(T(b), T(q), 1.0, rho, 7, z=z, theta=th, want_resid=True, adaptive=True)
    sched = np.concatenate([N(r1)[:, :, 2], N(r2)[:, :, 2], N(rho)[None]])
    ref = dct.code(b, q, 1.0, 10.0, 14, rho_schedule=sched)
    assert np.abs(N(z) - ref["z"]).max() <= CODE_TOL
    assert np.abs(N(th) - ref["theta"]).max() <= CODE_TOL


def test_dct_rejects_unsupported(lib):
    import torch
    with pytest.raises(lib.DualCSCError):   # 256 x 256 is beyond one tile
        lib.code_dct(torch.zeros((1, 1, 256, 256), device="cuda"), torch.zeros((2, 1, 3, 3), device="cuda"),
                     1.0, 1.0, 2)
    with pytest.raises(lib.DualCSCError):   # quadrant wider than 16
        lib.code_dct(torch.zeros((1, 1, 64, 64), device="cuda"), torch.zeros((2, 1, 3, 17), device="cuda"),
                     1.0, 1.0, 2)
