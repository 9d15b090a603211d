"""csc_code_noalloc (the entry point for callers that cannot allocate device
memory) against csc_code through the C ABI: two calls in a row, the second
on a smaller problem, each equal to csc_code's result bit for bit (same
kernels, same inputs, fixed-order reductions) and within the contract of the
FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tolerances import CODE_TOL

pytestmark = pytest.mark.gpu


def _call_both(lib, b, d, beta, rho, iters, adaptive):
    import torch
    dc = lib
    so = dc.load()
    bt = torch.from_numpy(b).cuda()
    dt = torch.from_numpy(d).cuda()
    N, K = b.shape[0], d.shape[0]
    shape = dc.Shape.make(N, b.shape[1], K, b.shape[2:], d.shape[2:])
    flags = dc.Z_ZERO | dc.THETA_ZERO | (dc.ADAPTIVE_RHO if adaptive else 0)
    out = []
    for noalloc in (False, True):
        z = torch.full((N, K) + b.shape[2:], float("nan"), dtype=torch.float32, device="cuda")
        th = torch.full_like(z, float("nan"))
        rho_t = torch.full((N,), float(rho), dtype=torch.float32, device="cuda")
        resid = torch.empty((iters, N, 3), dtype=torch.float64, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        if noalloc:
            rc = so.csc_code_noalloc(ctypes.byref(shape), bt.data_ptr(), dt.data_ptr(), float(beta), rho_t.data_ptr(),
                                     int(iters), flags, z.data_ptr(), th.data_ptr(), resid.data_ptr(), st)
        else:
            nbytes = so.csc_workspace_bytes(ctypes.byref(shape), dc.OP_CODE, flags)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = ws.data_ptr() + (-ws.data_ptr()) % 256
            rc = so.csc_code(ctypes.byref(shape), bt.data_ptr(), dt.data_ptr(), float(beta), rho_t.data_ptr(),
                             int(iters), flags, z.data_ptr(), th.data_ptr(), resid.data_ptr(), base, nbytes, st)
        assert rc == 0, so.csc_strerror(rc)
        torch.cuda.synchronize()
        out.append((z.cpu().numpy(), th.cpu().numpy(), rho_t.cpu().numpy(), resid.cpu().numpy()))
    return out


def test_noalloc_equals_csc_code_twice(lib):
    # first call: the 4 x 64^2, K = 16 workload with adaptive rho
    cfg = synth.CONFIGS["small"]
    b, d = synth.make_inputs(cfg)
    print("noalloc call 1: 4 x 64^2, K=16, adaptive rho", flush=True)
    (z0, t0, r0, s0), (z1, t1, r1, s1) = _call_both(lib, b, d, cfg.beta, cfg.rho, cfg.t_in, True)
    assert np.array_equal(z0, z1) and np.array_equal(t0, t1)
    assert np.array_equal(r0, r1) and np.array_equal(s0, s1)
    assert np.count_nonzero(z1) / z1.size > 0.01
    # second call, smaller: 2 images 32 x 32, K = 5 (odd: a half-empty pair), fixed rho
    b2 = np.ascontiguousarray(b[:2, :, :32, :32]) * np.float32(1.5)
    d2 = synth.unit_filters(5, 1, (7, 7), 77)
    print("noalloc call 2: 2 x 32^2, K=5, fixed rho", flush=True)
    (z0, t0, r0, s0), (z1, t1, r1, s1) = _call_both(lib, b2, d2, cfg.beta, cfg.rho, 15, False)
    assert np.array_equal(z0, z1) and np.array_equal(t0, t1)
    assert np.array_equal(s0, s1)
    ref = oracle.code(b2, d2, cfg.beta, cfg.rho, 15)
    assert np.count_nonzero(ref["z"]) / ref["z"].size > 0.01
    assert np.abs(z1 - ref["z"]).max() <= CODE_TOL


def test_noalloc_rejects_oversized_problem(lib):
    import torch
    so = lib.load()
    shape = lib.Shape.make(16, 1, 100, (256, 256), (11, 11))
    assert so.csc_workspace_bytes(ctypes.byref(shape), lib.OP_CODE, 0) > lib.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(1, device="cuda")
    rc = so.csc_code_noalloc(ctypes.byref(shape), x.data_ptr(), x.data_ptr(), 1.0, x.data_ptr(), 1, 0,
                             x.data_ptr(), None, None, torch.cuda.current_stream().cuda_stream)
    assert rc == lib.ESCRATCH
