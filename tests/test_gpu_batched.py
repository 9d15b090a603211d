"""Batched ragged coding (csc_code_batched) on the GPU: per-image parity with
the FP64 oracle, bitwise equality with the plain per-class solver, hipGraph
replays equal to the eager call, and the autotuner's table."""
import numpy as np
import pytest

import oracle
import synth
from tolerances import code_tol

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def ragged_case(n=10, k=6, lo=20, hi=140, seed=5):
    rng = np.random.default_rng(seed)
    imgs = []
    for _ in range(n):
        h, w = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        f = synth.contrast_normalize(synth.one_over_f(rng, (h, w))) * 30.0
        g = (synth.next_pow2(max(h, 8)), synth.next_pow2(max(w, 8)))
        pad = np.zeros(g, np.float32)
        pad[:h, :w] = f
        imgs.append(pad[None])
    d = synth.unit_filters(k, 1, (11, 11), seed + 1)
    return imgs, d


def test_batched_matches_oracle(lib):
    imgs, d = ragged_case()
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    assert len(pb.classes((11, 11))) >= 3
    z = pb.z_views(lib.code_batched(pb, T(d), 1.0, 10.0, 12, graph=False))
    dens = []
    for im, zg in zip(imgs, z):
        ref = oracle.code(im[None], d, 1.0, 10.0, 12)["z"][0]
        dens.append(np.count_nonzero(ref) / ref.size)
        assert np.abs(zg.cpu().numpy() - ref).max() <= code_tol(ref)
    assert np.mean(dens) > 0.005


def test_batched_equals_plain_per_class(lib):
    import torch
    imgs, d = ragged_case(n=9, seed=9)
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    zb = pb.z_views(lib.code_batched(pb, T(d), 1.0, 10.0, 8, graph=False))
    by_class = {}
    for i, im in enumerate(imgs):
        by_class.setdefault(im.shape[1:], []).append(i)
    for g, idx in by_class.items():
        bt = T(np.stack([imgs[i] for i in idx]))
        zp, _, _, _ = lib.code(bt, T(d), 1.0, 10.0, 8)
        for r, i in enumerate(idx):
            assert torch.equal(zp[r], zb[i]), (g, i)


def test_batched_graph_replay_equals_eager(lib):
    import torch
    imgs, d = ragged_case(n=8, seed=13)
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    dt = T(d)
    z_eager = lib.code_batched(pb, dt, 1.0, 10.0, 6, graph=False).clone()
    zbuf = torch.empty_like(z_eager)
    other = T(np.stack([imgs[0]] * 2))
    for rep in range(3):
        zbuf.fill_(123.0)
        lib.code_batched(pb, dt, 1.0, 10.0, 6, z=zbuf, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(zbuf, z_eager), rep
        lib.code(other, dt, 1.0, 10.0, 3)        # unrelated eager work between replays
        torch.cuda.synchronize()


def test_batched_autotune_table(lib, tmp_path, monkeypatch):
    monkeypatch.setenv("DUALCSC_TUNE_FILE", str(tmp_path / "tune.json"))
    imgs, d = ragged_case(n=6, k=8, seed=17)
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    dt = T(d)
    ppg = lib.autotune_batched(pb, dt, 1.0, 10.0, iters=2)
    cls = pb.classes((11, 11))
    assert len(ppg) == len(cls) and all(1 <= v <= 4 for v in ppg)
    assert lib.load_tuning(pb, (11, 11)) is not None
    z = pb.z_views(lib.code_batched(pb, dt, 1.0, 10.0, 8, graph=False))
    for im, zg in zip(imgs, z):
        ref = oracle.code(im[None], d, 1.0, 10.0, 8)["z"][0]
        assert np.abs(zg.cpu().numpy() - ref).max() <= code_tol(ref)


def test_batched_rejects_bad_tables(lib):
    import ctypes
    imgs, d = ragged_case(n=3, seed=21)
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    bt = pb.struct((11, 11))
    bt.k = 0
    assert lib.load().csc_batch_workspace_bytes(ctypes.byref(bt)) == 0


def test_batched_autotune_stays_in_workspace(lib):
    """The autotuner times each class alone with candidate groupings; one
    with fewer pairs per group needs more partial spectra than the batch's
    own layout gives that class.  Every candidate must stay inside the
    workspace the batch asks for: a guard region after it is unchanged.
    (3 images 256x256 with K = 64 default to two pairs per group, so one
    pair per group would need twice the class's partial spectra.)"""
    import ctypes
    import torch
    rng = np.random.default_rng(23)
    imgs = [(synth.contrast_normalize(synth.one_over_f(rng, (256, 256))) * 30.0)[None].astype(np.float32)
            for _ in range(3)]
    imgs.append((synth.contrast_normalize(synth.one_over_f(rng, (64, 64))) * 30.0)[None].astype(np.float32))
    d = synth.unit_filters(64, 1, (11, 11), 24)
    pb = lib.PackedBatch([T(im) for im in imgs], d.shape[0])
    so = lib.load()
    bt = pb.struct((11, 11))
    need = so.csc_batch_workspace_bytes(ctypes.byref(bt))
    guard = 64 << 20
    buf = torch.full((need + 256 + guard,), 0x5A, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    start = base - buf.data_ptr() + need
    z = torch.empty(pb.z_numel, dtype=torch.float32, device="cuda")
    ncls = len(pb.classes((11, 11)))
    out = (ctypes.c_int32 * ncls)()
    rc = so.csc_batch_autotune(ctypes.byref(bt), pb.b.data_ptr(), T(d).data_ptr(), 1.0, 10.0, 2, z.data_ptr(),
                               ctypes.c_void_p(base), need, torch.cuda.current_stream().cuda_stream, out, ncls)
    assert rc == 0, so.csc_strerror(rc)
    torch.cuda.synchronize()
    assert bool((buf[start:start + guard] == 0x5A).all())
    assert all(v >= 1 for v in out)
