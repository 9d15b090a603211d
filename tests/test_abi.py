"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, sizes workspaces, and rejects bad
arguments before anything is enqueued."""
import ctypes
import os
import re

import pytest

import paper_1709_09479_amd as dc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dualcsc.h")

pytestmark = pytest.mark.skipif(not os.path.exists(dc.lib_path()), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csc_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = dc.load()
    names = declared_functions()
    assert {"csc_code", "csc_learn", "csc_objective", "csc_workspace_bytes"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_and_strerror():
    lib = dc.load()
    assert lib.csc_abi_version() == dc.ABI_VERSION
    for code in (0, -1, -2, -3, -4, -99):
        assert isinstance(lib.csc_strerror(code), bytes)


def shape(n=2, j=1, k=4, grid=(64, 64), fsupp=(11, 11)):
    return dc.Shape.make(n, j, k, grid, fsupp)


@pytest.mark.parametrize("op", [dc.OP_CODE, dc.OP_LEARN, dc.OP_OBJECTIVE])
def test_workspace_sizes_positive_and_monotone(op):
    lib = dc.load()
    a = lib.csc_workspace_bytes(ctypes.byref(shape(n=2)), op, 0)
    b = lib.csc_workspace_bytes(ctypes.byref(shape(n=8)), op, 0)
    c = lib.csc_workspace_bytes(ctypes.byref(shape(n=2, grid=(128, 128))), op, 0)
    assert 0 < a < b and a < c


@pytest.mark.parametrize("bad", [
    dict(grid=(60, 64)),            # not a power of two
    dict(grid=(64, 64), fsupp=(65, 3)),  # support larger than grid
    dict(k=0), dict(n=0), dict(j=0), dict(j=4),
    dict(grid=(512, 512)),          # beyond the supported sides
    dict(grid=(4, 64)),
])
def test_invalid_shapes_have_no_workspace(bad):
    lib = dc.load()
    assert lib.csc_workspace_bytes(ctypes.byref(shape(**bad)), dc.OP_CODE, 0) == 0


def test_abi_version_mismatch_rejected():
    lib = dc.load()
    s = shape()
    s.abi_version = 99
    assert lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_CODE, 0) == 0


FAKE = 0x1000  # never dereferenced: every call below fails validation first


def test_code_argument_errors():
    lib = dc.load()
    s = shape()
    ws_need = lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_CODE, 0)
    call = lambda **kw: lib.csc_code(
        ctypes.byref(kw.get("s", s)), kw.get("b", FAKE), kw.get("d", FAKE), kw.get("beta", 1.0),
        kw.get("rho", FAKE), kw.get("iters", 5), kw.get("flags", 0), kw.get("z", FAKE), None, None,
        kw.get("ws", 0x100000), kw.get("wsb", ws_need), None)
    assert call(b=None) == dc.EINVAL
    assert call(d=None) == dc.EINVAL
    assert call(rho=None) == dc.EINVAL
    assert call(z=None) == dc.EINVAL
    assert call(beta=-1.0) == dc.EINVAL
    assert call(beta=float("nan")) == dc.EINVAL
    assert call(iters=-1) == dc.EINVAL
    assert call(flags=0x100) == dc.EINVAL
    assert call(ws=None) == dc.EWORKSPACE
    assert call(wsb=ws_need - 1) == dc.EWORKSPACE
    assert call(ws=0x100008) == dc.EWORKSPACE       # misaligned
    bad = shape(grid=(48, 64))
    assert call(s=bad) == dc.EINVAL
    assert call(s=shape(grid=(512, 64))) == dc.EUNSUPPORTED


def test_learn_and_objective_argument_errors():
    lib = dc.load()
    s = shape()
    need_l = lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_LEARN, 0)
    need_o = lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_OBJECTIVE, 0)
    L = lambda **kw: lib.csc_learn(ctypes.byref(s), FAKE, FAKE, kw.get("d", FAKE), kw.get("mu", FAKE), FAKE,
                                   kw.get("inner", 3), kw.get("cg", 3), kw.get("flags", 0), kw.get("ws", 0x100000),
                                   kw.get("wsb", need_l), None)
    assert L(d=None) == dc.EINVAL
    assert L(mu=None) == dc.EINVAL
    assert L(inner=0) == dc.EINVAL
    assert L(cg=-1) == dc.EINVAL
    assert L(flags=dc.ADAPTIVE_RHO) == dc.EINVAL
    assert L(flags=dc.LEARN_DIRECT | dc.LEARN_SPAN) == dc.EINVAL
    assert L(wsb=need_l - 1) == dc.EWORKSPACE
    O = lambda **kw: lib.csc_objective(ctypes.byref(s), FAKE, FAKE, FAKE, kw.get("beta", 1.0), kw.get("out", FAKE),
                                       0x100000, kw.get("wsb", need_o), None)
    assert O(out=None) == dc.EINVAL
    assert O(beta=-0.5) == dc.EINVAL
    assert O(wsb=0) == dc.EWORKSPACE


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    b = torch.zeros(1, 1, 16, 16)
    d = torch.zeros(2, 1, 3, 3)
    with pytest.raises(dc.DualCSCError):
        dc.code(b, d, 1.0, 1.0, 2)


def test_trace_argument_errors():
    """A negative sampling period is rejected before any HIP call; reading an
    unknown class or into NULL outputs is CSC_EINVAL."""
    lib = dc.load()
    assert lib.csc_trace_enable(-1) == -1
    ms, cnt = ctypes.c_double(), ctypes.c_int()
    assert lib.csc_trace_read(6, ctypes.byref(ms), ctypes.byref(cnt)) == -1
    assert lib.csc_trace_read(-1, ctypes.byref(ms), ctypes.byref(cnt)) == -1
    assert lib.csc_trace_read(0, None, ctypes.byref(cnt)) == -1
    with pytest.raises(ValueError):
        dc.trace_enable(True, every=0)


def test_tolerance_entry_point_argument_errors():
    """csc_code_tol / csc_learn_tol validate their stopping-rule arguments on
    the host before anything is enqueued (no GPU needed)."""
    lib = dc.load()
    s = shape()
    wc = lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_CODE, 0)
    code = lambda **kw: lib.csc_code_tol(
        ctypes.byref(s), FAKE, FAKE, 1.0, FAKE, kw.get("iters", 5), kw.get("tol", 1e-3), kw.get("flags", 0),
        FAKE, None, None, None, 0x100000, kw.get("wsb", wc), None)
    assert code(tol=0.0) == dc.EINVAL
    assert code(tol=-1.0) == dc.EINVAL
    assert code(tol=float("nan")) == dc.EINVAL
    assert code(tol=float("inf")) == dc.EINVAL
    assert code(iters=-1) == dc.EINVAL
    assert code(flags=dc.USE_GRAPH) == dc.EINVAL
    assert code(wsb=wc - 1) == dc.EWORKSPACE
    wl = lib.csc_workspace_bytes(ctypes.byref(s), dc.OP_LEARN, 0)
    learn = lambda **kw: lib.csc_learn_tol(
        ctypes.byref(s), FAKE, FAKE, FAKE, FAKE, FAKE, kw.get("inner", 2), kw.get("cg", 5), kw.get("tol", 1e-3),
        kw.get("flags", 0), None, 0x100000, kw.get("wsb", wl), None)
    assert learn(tol=-1e-3) == dc.EINVAL
    assert learn(tol=float("nan")) == dc.EINVAL
    assert learn(inner=0) == dc.EINVAL
    assert learn(cg=-1) == dc.EINVAL
    assert learn(flags=dc.USE_GRAPH) == dc.EINVAL
    assert learn(wsb=wl - 1) == dc.EWORKSPACE


def test_unrolled_record_size():
    """A checkpoint record holds z and theta ([N][K][grid] each) and the
    solver's spectral state (three [N][1][grid] complex arrays); J > 1 has no
    differentiable form."""
    lib = dc.load()
    for n, k, grid in ((2, 4, (64, 64)), (3, 7, (32, 128)), (1, 100, (256, 256))):
        s = shape(n=n, k=k, grid=grid)
        assert lib.csc_unrolled_record_floats(ctypes.byref(s)) == n * grid[0] * grid[1] * (2 * k + 6)
    assert lib.csc_unrolled_record_floats(ctypes.byref(shape(j=3))) == 0
    assert lib.csc_unrolled_record_floats(ctypes.byref(shape(grid=(60, 64)))) == 0


def test_check_finite_argument_errors():
    """csc_check_finite validates its arguments on the host; CSC_ENONFINITE
    has its own message."""
    lib = dc.load()
    assert lib.csc_check_finite(None, 4, FAKE, None) == dc.EINVAL
    assert lib.csc_check_finite(FAKE, -1, FAKE, None) == dc.EINVAL
    assert lib.csc_check_finite(FAKE, 4, None, None) == dc.EINVAL
    assert b"non-finite" in lib.csc_strerror(dc.ENONFINITE)


def test_noalloc_rejects_before_enqueue():
    """csc_code_noalloc validates like csc_code and refuses a problem whose
    scratch exceeds its static array before touching the device."""
    lib = dc.load()
    big = shape(n=16, k=100, grid=(256, 256))
    assert lib.csc_workspace_bytes(ctypes.byref(big), dc.OP_CODE, 0) > dc.NOALLOC_SCRATCH_BYTES
    call = lambda s, **kw: lib.csc_code_noalloc(
        ctypes.byref(s), kw.get("b", FAKE), FAKE, kw.get("beta", 1.0), FAKE, kw.get("iters", 5),
        kw.get("flags", 0), FAKE, None, None, None)
    assert call(big) == dc.ESCRATCH
    assert call(shape(), b=None) == dc.EINVAL
    assert call(shape(), beta=-1.0) == dc.EINVAL
    assert call(shape(), iters=-1) == dc.EINVAL
    assert call(shape(), flags=dc.USE_GRAPH) == dc.EINVAL
    assert call(shape(grid=(60, 64))) == dc.EINVAL
    assert b"64 MiB" in lib.csc_strerror(dc.ESCRATCH)
