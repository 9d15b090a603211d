"""Python binding of libdualcsc (dual-domain convolutional sparse coding on
MI355X).  Argument marshalling only: every step runs in the HIP library;
torch tensors provide device memory and the stream.

    import paper_1709_09479_amd as dc
    z, theta, resid = dc.code(b, d, beta=1.0, rho=10.0, iters=20)
    d, mu, gamma = dc.learn(b, z, fsupp=(11, 11), mu=mu, gamma=gamma)
    per_image, total = dc.objective(b, d, z, beta=1.0)

Shapes follow the C header ``include/dualcsc.h``: images b [N][J][*grid],
filters d [K][J][*fsupp], codes z [N][K][*grid], all float32 on the GPU.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence, Tuple

__all__ = [
    "DualCSCError", "load", "lib_path", "Shape", "code", "learn", "objective",
    "learn_dictionary", "workspace_bytes", "trace_enable", "trace_read", "ADAPTIVE_RHO", "Z_ZERO", "THETA_ZERO",
    "GAMMA_ZERO", "USE_GRAPH", "PackedBatch", "code_batched", "autotune_batched", "unrolled_code", "csc_loss",
    "code_until", "learn_until", "code_dct", "objective_dct", "NUCLEAR",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libdualcsc.so"

ABI_VERSION = 2
OK, EINVAL, EWORKSPACE, EUNSUPPORTED, EHIP, ENONFINITE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 64 << 20
OP_CODE, OP_LEARN, OP_OBJECTIVE, OP_DCT = 1, 2, 3, 4
ADAPTIVE_RHO, Z_ZERO, THETA_ZERO, GAMMA_ZERO, USE_GRAPH, NUCLEAR = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
LEARN_DIRECT, LEARN_SPAN = 0x40, 0x80
_REG_FLAGS = {"l1": 0, "nuclear": NUCLEAR}


def _reg_flag(reg: str) -> int:
    if reg not in _REG_FLAGS:
        raise DualCSCError(EINVAL, "reg must be 'l1' or 'nuclear'")
    return _REG_FLAGS[reg]


class DualCSCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("j", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("ndim", ctypes.c_int32),
        ("grid", ctypes.c_int32 * 3),
        ("fsupp", ctypes.c_int32 * 3),
    ]

    @classmethod
    def make(cls, n: int, j: int, k: int, grid: Sequence[int], fsupp: Sequence[int]) -> "Shape":
        s = cls()
        s.abi_version = ABI_VERSION
        s.n, s.j, s.k = int(n), int(j), int(k)
        s.ndim = len(grid)
        for a in range(3):
            s.grid[a] = int(grid[a]) if a < len(grid) else 0
            s.fsupp[a] = int(fsupp[a]) if a < len(fsupp) else 0
        return s


class Batch(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("fsupp", ctypes.c_int32 * 2),
        ("grid", ctypes.POINTER(ctypes.c_int32)),
        ("b_off", ctypes.POINTER(ctypes.c_int64)),
        ("z_off", ctypes.POINTER(ctypes.c_int64)),
        ("ppg", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def lib_path() -> str:
    """The in-tree library (built by ``paper_1709_09479_amd.build``)."""
    return os.path.join(_PKG, _LIB_NAME)


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raises if it is missing (there is no
    fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise DualCSCError(EHIP, "libdualcsc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, u32, f32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_float, ctypes.c_size_t
    sp = ctypes.POINTER(Shape)
    lib.csc_abi_version.restype = i32
    lib.csc_strerror.restype = ctypes.c_char_p
    lib.csc_strerror.argtypes = [i32]
    lib.csc_workspace_bytes.restype = sz
    lib.csc_workspace_bytes.argtypes = [sp, i32, u32]
    lib.csc_code.restype = i32
    lib.csc_code.argtypes = [sp, vp, vp, f32, vp, i32, u32, vp, vp, vp, vp, sz, vp]
    lib.csc_code_noalloc.restype = i32
    lib.csc_code_noalloc.argtypes = [sp, vp, vp, f32, vp, i32, u32, vp, vp, vp, vp]
    lib.csc_learn.restype = i32
    lib.csc_learn.argtypes = [sp, vp, vp, vp, vp, vp, i32, i32, u32, vp, sz, vp]
    lib.csc_code_tol.restype = i32
    lib.csc_code_tol.argtypes = [sp, vp, vp, f32, vp, i32, f32, u32, vp, vp, vp, vp, vp, sz, vp]
    lib.csc_learn_tol.restype = i32
    lib.csc_learn_tol.argtypes = [sp, vp, vp, vp, vp, vp, i32, i32, f32, u32, vp, vp, sz, vp]
    lib.csc_objective.restype = i32
    lib.csc_objective.argtypes = [sp, vp, vp, vp, f32, vp, vp, sz, vp]
    lib.csc_code_dct.restype = i32
    lib.csc_code_dct.argtypes = [sp, vp, vp, f32, vp, i32, u32, vp, vp, vp, vp, sz, vp]
    lib.csc_objective_dct.restype = i32
    lib.csc_objective_dct.argtypes = [sp, vp, vp, vp, f32, vp, vp, sz, vp]
    lib.csc_objective_reg.restype = i32
    lib.csc_objective_reg.argtypes = [sp, vp, vp, vp, f32, u32, vp, vp, sz, vp]
    lib.csc_trace_enable.restype = i32
    lib.csc_trace_enable.argtypes = [i32]
    lib.csc_check_finite.restype = i32
    lib.csc_check_finite.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.csc_trace_read.restype = i32
    lib.csc_trace_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    bp = ctypes.POINTER(Batch)
    lib.csc_batch_workspace_bytes.restype = sz
    lib.csc_batch_workspace_bytes.argtypes = [bp]
    lib.csc_batch_classes.restype = i32
    lib.csc_batch_classes.argtypes = [bp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), i32]
    lib.csc_code_batched.restype = i32
    lib.csc_code_batched.argtypes = [bp, vp, vp, f32, f32, i32, u32, vp, vp, sz, vp]
    lib.csc_batch_autotune.restype = i32
    lib.csc_batch_autotune.argtypes = [bp, vp, vp, f32, f32, i32, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_int32), i32]
    lib.csc_unrolled_workspace_bytes.restype = sz
    lib.csc_unrolled_workspace_bytes.argtypes = [sp, i32]
    lib.csc_unrolled_record_floats.restype = ctypes.c_int64
    lib.csc_unrolled_record_floats.argtypes = [sp]
    lib.csc_code_unrolled.restype = i32
    lib.csc_code_unrolled.argtypes = [sp, vp, vp, f32, vp, i32, i32, vp, vp, vp, sz, vp]
    lib.csc_code_backward.restype = i32
    lib.csc_code_backward.argtypes = [sp, vp, vp, f32, vp, i32, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.csc_loss_grad.restype = i32
    lib.csc_loss_grad.argtypes = [sp, vp, vp, vp, f32, vp, vp, vp, vp, vp, sz, vp]
    if lib.csc_abi_version() != ABI_VERSION:
        raise DualCSCError(EINVAL, "ABI version mismatch")
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != OK:
        msg = load().csc_strerror(rc).decode()
        raise DualCSCError(rc, msg)


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return _torch().cuda.current_stream().cuda_stream


_WS = {}


def _workspace(shape: Shape, op: int, flags: int, device):
    """Caller-side workspace (torch allocation), cached per device and size."""
    torch = _torch()
    nbytes = load().csc_workspace_bytes(ctypes.byref(shape), op, flags)
    if nbytes == 0:
        _check(EINVAL)
    key = (str(device), op, flags & NUCLEAR)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes + 256:
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        _WS[key] = buf
    base = buf.data_ptr()
    off = (-base) % 256
    return base + off, nbytes


def workspace_bytes(n, j, k, grid, fsupp, op=OP_CODE, flags=0) -> int:
    s = Shape.make(n, j, k, grid, fsupp)
    return int(load().csc_workspace_bytes(ctypes.byref(s), op, flags))


def _need(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise DualCSCError(EINVAL, "%s must be a contiguous float32 CUDA tensor" % name)


def _shape_of(b, d) -> Shape:
    nd = b.dim() - 2
    return Shape.make(b.shape[0], b.shape[1], d.shape[0], tuple(b.shape[2:]), tuple(d.shape[2:2 + nd]))


class _GraphStream:
    """Runs a library call on a non-default stream (graph capture is not
    possible on the NULL stream), ordered after and before the current one."""

    def __init__(self, enabled: bool):
        self.enabled = enabled

    def __enter__(self):
        torch = _torch()
        self.cur = torch.cuda.current_stream()
        if not self.enabled:
            return self.cur.cuda_stream
        global _SIDE_STREAM
        if self.cur.cuda_stream != 0:
            self.side = None
            return self.cur.cuda_stream
        if _SIDE_STREAM is None:
            _SIDE_STREAM = torch.cuda.Stream()
        self.side = _SIDE_STREAM
        self.side.wait_stream(self.cur)
        return self.side.cuda_stream

    def __exit__(self, *exc):
        if self.enabled and self.side is not None:
            self.cur.wait_stream(self.side)
        return False


_SIDE_STREAM = None


def code(b, d, beta: float, rho, iters: int, z=None, theta=None, adaptive: bool = False,
         want_theta: bool = False, want_resid: bool = False, graph: bool = False, reg: str = "l1"):
    """ADMM coding (eq:Inference_solution) for ``iters`` iterations.

    b [N][J][*grid], d [K][J][*fsupp]; rho: float or [N] tensor (updated in
    place when adaptive).  z / theta: warm starts (modified in place) or None
    (start from zero).  reg: "l1" (eq:CSC) or "nuclear" (beta sum_k ||z_k||_*,
    low-rank maps).  Returns (z, theta or None, resid [iters][N][3] or None,
    rho tensor)."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(d, "d")
    shape = _shape_of(b, d)
    N, K = b.shape[0], d.shape[0]
    dev = b.device
    flags = (ADAPTIVE_RHO if adaptive else 0) | _reg_flag(reg)
    if z is None:
        z = torch.empty((N, K) + tuple(b.shape[2:]), dtype=torch.float32, device=dev)
        flags |= Z_ZERO
    _need(z, "z")
    if theta is None and want_theta:
        theta = torch.empty_like(z)
        flags |= THETA_ZERO
    if theta is not None:
        _need(theta, "theta")
    if isinstance(rho, torch.Tensor):
        rho_t = rho
    else:
        rho_t = torch.full((N,), float(rho), dtype=torch.float32, device=dev)
    _need(rho_t, "rho")
    resid = torch.empty((iters, N, 3), dtype=torch.float64, device=dev) if (want_resid and iters > 0) else None
    ws, nbytes = _workspace(shape, OP_CODE, flags, dev)
    with _GraphStream(graph) as st:
        rc = lib.csc_code(ctypes.byref(shape), _ptr(b), _ptr(d), float(beta), _ptr(rho_t), int(iters),
                          flags | (USE_GRAPH if graph else 0), _ptr(z), _ptr(theta), _ptr(resid), ws, nbytes, st)
    _check(rc)
    return z, theta, resid, rho_t


def learn(b, z, fsupp: Sequence[int], mu=None, gamma=None, inner_iters: int = 10, cg_iters: int = 10,
          out=None, graph: bool = False, form: str = "auto"):
    """Dual dictionary learning (eq:Learning_gamma, eq:Learning_Solution,
    eq:mu_update).  Returns (d [K][J][*fsupp], mu [K], gamma [N][J][*grid]);
    mu and gamma are updated in place when given; ``out`` receives d.  With
    ``graph`` the call is captured once and replayed when called again with
    the same tensors.  ``form`` picks the CG's form: "auto" (the library's
    cost model), "direct" (the operator on the full CG vectors,
    CSC_LEARN_DIRECT) or "span" (the span form wherever the plan allows it,
    CSC_LEARN_SPAN)."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(z, "z")
    N, J, K = b.shape[0], b.shape[1], z.shape[1]
    dev = b.device
    fsupp = tuple(int(s) for s in fsupp)
    shape = Shape.make(N, J, K, tuple(b.shape[2:]), fsupp)
    flags = 0
    if mu is None:
        mu = torch.ones(K, dtype=torch.float32, device=dev)
    if gamma is None:
        gamma = torch.empty_like(b)
        flags |= GAMMA_ZERO
    _need(mu, "mu")
    _need(gamma, "gamma")
    d = out if out is not None else torch.empty((K, J) + fsupp, dtype=torch.float32, device=dev)
    _need(d, "out")
    ws, nbytes = _workspace(shape, OP_LEARN, flags, dev)
    if form not in ("auto", "direct", "span"):
        raise ValueError("form must be 'auto', 'direct' or 'span'")
    flags |= {"auto": 0, "direct": LEARN_DIRECT, "span": LEARN_SPAN}[form]
    with _GraphStream(graph) as st:
        rc = lib.csc_learn(ctypes.byref(shape), _ptr(b), _ptr(z), _ptr(d), _ptr(mu), _ptr(gamma),
                           int(inner_iters), int(cg_iters), flags | (USE_GRAPH if graph else 0), ws, nbytes, st)
    _check(rc)
    return d, mu, gamma


def code_until(b, d, beta: float, rho, max_iters: int, tol: float, z=None, theta=None, adaptive: bool = False,
               want_theta: bool = False, want_resid: bool = False, reg: str = "l1"):
    """ADMM coding until every image's RMS primal and dual residuals are at
    most ``tol`` (at most ``max_iters`` iterations; the decision is taken on
    the device).  Returns (z, theta or None, resid [done][N][3] or None, rho
    tensor, done)."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(d, "d")
    shape = _shape_of(b, d)
    N, K = b.shape[0], d.shape[0]
    dev = b.device
    flags = (ADAPTIVE_RHO if adaptive else 0) | _reg_flag(reg)
    if z is None:
        z = torch.empty((N, K) + tuple(b.shape[2:]), dtype=torch.float32, device=dev)
        flags |= Z_ZERO
    _need(z, "z")
    if theta is None and want_theta:
        theta = torch.empty_like(z)
        flags |= THETA_ZERO
    if theta is not None:
        _need(theta, "theta")
    rho_t = rho if isinstance(rho, torch.Tensor) else torch.full((N,), float(rho), dtype=torch.float32, device=dev)
    _need(rho_t, "rho")
    resid = torch.empty((max_iters, N, 3), dtype=torch.float64, device=dev) if (want_resid and max_iters > 0) else None
    done = torch.zeros(1, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(shape, OP_CODE, flags, dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    _check(lib.csc_code_tol(ctypes.byref(shape), _ptr(b), _ptr(d), float(beta), _ptr(rho_t), int(max_iters),
                            float(tol), flags, _ptr(z), _ptr(theta), _ptr(resid), _ptr(done), ws, nbytes,
                            ctypes.c_void_p(st)))
    n_done = int(done.item())
    return z, theta, (resid[:n_done] if resid is not None else None), rho_t, n_done


def learn_until(b, z, fsupp: Sequence[int], mu=None, gamma=None, inner_iters: int = 10, max_cg: int = 10,
                cg_tol: float = 1e-3, out=None):
    """Dual dictionary learning whose CG solves stop once every channel's
    residual is at most ``cg_tol`` times its right-hand side.  Returns (d,
    mu, gamma, CG steps per multiplier update as a list)."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(z, "z")
    N, J, K = b.shape[0], b.shape[1], z.shape[1]
    dev = b.device
    fsupp = tuple(int(s) for s in fsupp)
    shape = Shape.make(N, J, K, tuple(b.shape[2:]), fsupp)
    flags = 0
    if mu is None:
        mu = torch.ones(K, dtype=torch.float32, device=dev)
    if gamma is None:
        gamma = torch.empty_like(b)
        flags |= GAMMA_ZERO
    _need(mu, "mu")
    _need(gamma, "gamma")
    d = out if out is not None else torch.empty((K, J) + fsupp, dtype=torch.float32, device=dev)
    _need(d, "out")
    counts = torch.zeros(inner_iters, dtype=torch.int32, device=dev)
    ws, nbytes = _workspace(shape, OP_LEARN, flags, dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    _check(lib.csc_learn_tol(ctypes.byref(shape), _ptr(b), _ptr(z), _ptr(d), _ptr(mu), _ptr(gamma), int(inner_iters),
                             int(max_cg), float(cg_tol), flags, _ptr(counts), ws, nbytes, ctypes.c_void_p(st)))
    return d, mu, gamma, [int(c) for c in counts.cpu()]


def objective(b, d, z, beta: float, reg: str = "l1"):
    """eq:CSC objective (with reg="nuclear" the regulariser is the nuclear
    norm of each map): returns a float64 tensor [N + 1] (per image, total)."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(d, "d")
    _need(z, "z")
    shape = _shape_of(b, d)
    flags = _reg_flag(reg)
    out = torch.empty(b.shape[0] + 1, dtype=torch.float64, device=b.device)
    ws, nbytes = _workspace(shape, OP_OBJECTIVE, flags, b.device)
    if flags:
        rc = lib.csc_objective_reg(ctypes.byref(shape), _ptr(b), _ptr(d), _ptr(z), float(beta), flags, _ptr(out), ws,
                                   nbytes, _stream())
    else:
        rc = lib.csc_objective(ctypes.byref(shape), _ptr(b), _ptr(d), _ptr(z), float(beta), _ptr(out), ws, nbytes,
                               _stream())
    _check(rc)
    return out


def code_dct(b, q, beta: float, rho, iters: int, z=None, theta=None, adaptive: bool = False,
             want_theta: bool = False, want_resid: bool = False):
    """Coding with symmetric boundaries (the DCT-domain variant, csc_code_dct):
    b [N][J][H][W]; q [K][J][M1][M2] quadrants of whole-sample symmetric
    filters (h[m1][m2] = q[|m1|][|m2|]).  Other arguments and results as
    code()."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(q, "q")
    shape = _shape_of(b, q)
    N, K = b.shape[0], q.shape[0]
    dev = b.device
    flags = ADAPTIVE_RHO if adaptive else 0
    if z is None:
        z = torch.empty((N, K) + tuple(b.shape[2:]), dtype=torch.float32, device=dev)
        flags |= Z_ZERO
    _need(z, "z")
    if theta is None and want_theta:
        theta = torch.empty_like(z)
        flags |= THETA_ZERO
    if theta is not None:
        _need(theta, "theta")
    rho_t = rho if isinstance(rho, torch.Tensor) else torch.full((N,), float(rho), dtype=torch.float32, device=dev)
    _need(rho_t, "rho")
    resid = torch.empty((iters, N, 3), dtype=torch.float64, device=dev) if (want_resid and iters > 0) else None
    ws, nbytes = _workspace(shape, OP_DCT, 0, dev)
    _check(lib.csc_code_dct(ctypes.byref(shape), _ptr(b), _ptr(q), float(beta), _ptr(rho_t), int(iters), flags,
                            _ptr(z), _ptr(theta), _ptr(resid), ws, nbytes, _stream()))
    return z, theta, resid, rho_t


def objective_dct(b, q, z, beta: float):
    """Objective of the symmetric-boundary problem: float64 tensor [N + 1]."""
    torch = _torch()
    lib = load()
    _need(b, "b")
    _need(q, "q")
    _need(z, "z")
    shape = _shape_of(b, q)
    out = torch.empty(b.shape[0] + 1, dtype=torch.float64, device=b.device)
    ws, nbytes = _workspace(shape, OP_DCT, 0, b.device)
    _check(lib.csc_objective_dct(ctypes.byref(shape), _ptr(b), _ptr(q), _ptr(z), float(beta), _ptr(out), ws, nbytes,
                                 _stream()))
    return out


TRACE_CODE_MAPS, TRACE_CODE_SPEC, TRACE_LEARN_A, TRACE_LEARN_B = 0, 1, 2, 3
TRACE_LEARN_SPAN_ROWS, TRACE_LEARN_SPAN_APPLY = 4, 5


def check_finite(*tensors) -> None:
    """Raise DualCSCError(ENONFINITE) if any of the given float32 device
    tensors holds a NaN or an infinity (csc_check_finite; waits for the
    stream)."""
    torch = _torch()
    lib = load()
    flags = torch.empty(max(1, len(tensors)), dtype=torch.int32, device=tensors[0].device if tensors else "cuda")
    for i, t in enumerate(tensors):
        _need(t, "tensor")
        _check(lib.csc_check_finite(_ptr(t), t.numel(), flags[i:].data_ptr(), _stream()))
    if tensors and int(flags[:len(tensors)].max().item()):
        raise DualCSCError(ENONFINITE, lib.csc_strerror(ENONFINITE).decode())


def trace_enable(on: bool = True, every: int = 1) -> None:
    """Start (clearing earlier records) or stop event tracing of launches;
    with ``every`` = n only every n-th launch of each class is bracketed."""
    if every < 1:
        raise ValueError("every must be >= 1")
    _check(load().csc_trace_enable(int(every) if on else 0))


def trace_read(cls: int) -> Tuple[float, int]:
    """(summed milliseconds, number of records) of a traced kernel class."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int(0)
    _check(load().csc_trace_read(int(cls), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def learn_dictionary(b, d0, beta: float, rho, t_in: int, t_out: int, inner_iters: int = 10,
                     cg_iters: int = 10, adaptive: bool = False, log_objective: bool = True, tau=None, tol=None,
                     cg_tol=None, reg: str = "l1"):
    """Alg. 1: alternate coding (warm-started z, theta) and learning
    (warm-started gamma, carried mu) for ``t_out`` outer steps.  Returns a dict
    with d, z, theta, mu, gamma, rho, the objective after each half step
    (float64 device tensors) and the number of outer steps taken.

    Convergence-driven mode: ``tau`` stops the alternation after the first
    outer step whose objective (after learning) changed by at most tau
    relative to the previous step's (this reads the objective back each
    step); ``tol`` and ``cg_tol`` are the stopping rules of code_until and
    learn_until (then ``t_in`` and ``cg_iters`` are the largest counts, and
    the counts taken are returned under "coding_iters" and "cg_counts").
    ``reg`` selects the regulariser of the coding steps and the objective."""
    torch = _torch()
    N, K = b.shape[0], d0.shape[0]
    d = d0.clone()
    fsupp = tuple(d0.shape[2:])
    z = theta = gamma = None
    mu = torch.ones(K, dtype=torch.float32, device=b.device)
    rho_t = rho if isinstance(rho, torch.Tensor) else torch.full((N,), float(rho), dtype=torch.float32,
                                                                 device=b.device)
    objs, code_its, cg_counts = [], [], []
    log_objective = log_objective or tau is not None
    steps = 0
    for _ in range(t_out):
        if tol is not None:
            z, theta, _, rho_t, n = code_until(b, d, beta, rho_t, t_in, tol, z=z, theta=theta, adaptive=adaptive,
                                                want_theta=True, reg=reg)
            code_its.append(n)
        else:
            z, theta, _, rho_t = code(b, d, beta, rho_t, t_in, z=z, theta=theta, adaptive=adaptive, want_theta=True,
                                      reg=reg)
        if log_objective:
            objs.append(objective(b, d, z, beta, reg)[-1:].clone())
        if cg_tol is not None:
            d, mu, gamma, c = learn_until(b, z, fsupp, mu, gamma, inner_iters, cg_iters, cg_tol)
            cg_counts.append(c)
        else:
            d, mu, gamma = learn(b, z, fsupp, mu, gamma, inner_iters, cg_iters)
        if log_objective:
            objs.append(objective(b, d, z, beta, reg)[-1:].clone())
        steps += 1
        if tau is not None and len(objs) >= 4:
            f_new, f_old = float(objs[-1].item()), float(objs[-3].item())
            if not (math.isfinite(f_new) and math.isfinite(f_old)):
                raise DualCSCError(ENONFINITE, load().csc_strerror(ENONFINITE).decode())
            if abs(f_new - f_old) <= tau * abs(f_old):
                break
    out = {"d": d, "z": z, "theta": theta, "mu": mu, "gamma": gamma, "rho": rho_t,
           "objectives": torch.cat(objs) if objs else None, "steps": steps}
    if tol is not None:
        out["coding_iters"] = code_its
    if cg_tol is not None:
        out["cg_counts"] = cg_counts
    return out


# ------------------------------------------------------------------ batched

class PackedBatch:
    """Images of uneven padded grids packed into one device buffer.

    ``b`` holds image i's H_i x W_i block at ``b_off[i]``; the codes of image
    i (K x H_i x W_i) live at ``z_off[i]`` of a buffer of ``z_numel``."""

    def __init__(self, images, k: int):
        torch = _torch()
        self.k = int(k)
        self.grids = [tuple(int(s) for s in im.shape[-2:]) for im in images]
        sizes = [h * w for h, w in self.grids]
        self.b_off, self.z_off = [], []
        ob = oz = 0
        for sz_ in sizes:
            self.b_off.append(ob)
            self.z_off.append(oz)
            ob += sz_
            oz += self.k * sz_
        self.z_numel = oz
        dev = images[0].device
        self.b = torch.cat([im.reshape(-1) for im in images]).to(dev).contiguous()
        n = len(images)
        self._grid = (ctypes.c_int32 * (2 * n))(*[v for g in self.grids for v in g])
        self._boff = (ctypes.c_int64 * n)(*self.b_off)
        self._zoff = (ctypes.c_int64 * n)(*self.z_off)
        self._ppg = None

    def struct(self, fsupp, ppg=None) -> Batch:
        bt = Batch()
        bt.abi_version = ABI_VERSION
        bt.n = len(self.grids)
        bt.k = self.k
        bt.fsupp[0], bt.fsupp[1] = int(fsupp[0]), int(fsupp[1])
        bt.grid = self._grid
        bt.b_off = self._boff
        bt.z_off = self._zoff
        if ppg is not None:
            self._ppg = (ctypes.c_int32 * len(ppg))(*[int(v) for v in ppg])
            bt.ppg = self._ppg
        return bt

    def classes(self, fsupp):
        bt = self.struct(fsupp)
        lib = load()
        nc = lib.csc_batch_classes(ctypes.byref(bt), None, None, 0)
        _check(0 if nc >= 0 else nc)
        g = (ctypes.c_int32 * (2 * nc))()
        c = (ctypes.c_int32 * nc)()
        lib.csc_batch_classes(ctypes.byref(bt), g, c, nc)
        return [((g[2 * i], g[2 * i + 1]), c[i]) for i in range(nc)]

    def z_views(self, z):
        """Per-image [K][H][W] views of a packed code buffer."""
        return [z[o:o + self.k * h * w].view(self.k, h, w) for o, (h, w) in zip(self.z_off, self.grids)]


def _tune_file():
    return os.environ.get("DUALCSC_TUNE_FILE") or os.path.join(
        os.path.expanduser("~"), ".cache", "dualcsc", "autotune.json")


def _tune_key(grid, count, k, fsupp):
    return "gfx950|%dx%d|n%d|k%d|f%dx%d" % (grid[0], grid[1], count, k, fsupp[0], fsupp[1])


def load_tuning(pb: PackedBatch, fsupp):
    """ppg table for the batch's classes from the persisted autotune file
    (None entries -> 0 = built-in choice)."""
    import json
    path = _tune_file()
    try:
        with open(path) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return None
    vals = [int(table.get(_tune_key(g, c, pb.k, fsupp), 0)) for g, c in pb.classes(fsupp)]
    return vals if any(vals) else None


def autotune_batched(pb: PackedBatch, d, beta: float, rho: float, iters: int = 3, persist: bool = True):
    """Measure the best filter pairs per workgroup for every single-tile grid
    class of the batch and (optionally) store them in the autotune file."""
    import json
    torch = _torch()
    lib = load()
    fsupp = tuple(d.shape[2:4])
    bt = pb.struct(fsupp)
    need = lib.csc_batch_workspace_bytes(ctypes.byref(bt))
    ws, nbytes = _workspace_raw(need, "batch", pb.b.device)
    z = torch.empty(pb.z_numel, dtype=torch.float32, device=pb.b.device)
    cls = pb.classes(fsupp)
    out = (ctypes.c_int32 * len(cls))()
    rc = lib.csc_batch_autotune(ctypes.byref(bt), _ptr(pb.b), _ptr(d), float(beta), float(rho), int(iters),
                                _ptr(z), ws, nbytes, _stream(), out, len(cls))
    _check(rc)
    ppg = [int(v) for v in out]
    if persist:
        path = _tune_file()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
        for (g, c), v in zip(cls, ppg):
            table[_tune_key(g, c, pb.k, fsupp)] = v
        with open(path, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return ppg


def _workspace_raw(nbytes, tag, device):
    torch = _torch()
    if nbytes == 0:
        _check(EINVAL)
    key = (str(device), tag)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes + 256:
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        _WS[key] = buf
    base = buf.data_ptr()
    return base + (-base) % 256, nbytes


def code_batched(pb: PackedBatch, d, beta: float, rho: float, iters: int, z=None, warm: bool = False,
                 graph: bool = True, ppg=None, stream=None):
    """Code every image of a PackedBatch (csc_code_batched).  Returns the
    packed codes (see PackedBatch.z_views); ``z`` is the output buffer, read
    as a warm start only when ``warm``.  ``ppg``: per-class pairs per
    workgroup (default: the persisted autotune table, else built-in).
    With ``graph`` the call is captured once and replayed on later calls with
    the same buffers; it runs on ``stream`` (a torch.cuda.Stream, default: a
    stream owned by this module) ordered after the current stream."""
    torch = _torch()
    lib = load()
    _need(d, "d")
    fsupp = tuple(d.shape[2:4])
    if ppg is None:
        ppg = load_tuning(pb, fsupp)
    bt = pb.struct(fsupp, ppg)
    need = lib.csc_batch_workspace_bytes(ctypes.byref(bt))
    ws, nbytes = _workspace_raw(need, "batch", pb.b.device)
    flags = 0 if warm else Z_ZERO
    if z is None:
        z = torch.empty(pb.z_numel, dtype=torch.float32, device=pb.b.device)
        flags = Z_ZERO
    _need(z, "z")
    cur = torch.cuda.current_stream()
    if graph:
        global _BATCH_STREAM
        s = stream or _BATCH_STREAM
        if s is None:
            s = _BATCH_STREAM = torch.cuda.Stream()
        s.wait_stream(cur)
        rc = lib.csc_code_batched(ctypes.byref(bt), _ptr(pb.b), _ptr(d), float(beta), float(rho), int(iters),
                                  flags | USE_GRAPH, _ptr(z), ws, nbytes, s.cuda_stream)
        cur.wait_stream(s)
    else:
        rc = lib.csc_code_batched(ctypes.byref(bt), _ptr(pb.b), _ptr(d), float(beta), float(rho), int(iters),
                                  flags, _ptr(z), ws, nbytes, cur.cuda_stream)
    _check(rc)
    return z


_BATCH_STREAM = None


# ----------------------------------------------------------- differentiable

def _diff_ws(shape, every, device):
    need = load().csc_unrolled_workspace_bytes(ctypes.byref(shape), int(every))
    return _workspace_raw(need, "diff", device)


def _rho_tensor(rho, n, device):
    torch = _torch()
    if isinstance(rho, torch.Tensor):
        return rho.to(device=device, dtype=torch.float32).contiguous()
    return torch.full((n,), float(rho), dtype=torch.float32, device=device)


def _make_unrolled():
    torch = _torch()

    class CSCUnrolled(torch.autograd.Function):
        """z^T = unrolled coding solve (csc_code_unrolled); the backward pass
        is the library's adjoint (csc_code_backward) with respect to the
        filters d and the sparsity weight beta (a tensor)."""

        @staticmethod
        def forward(ctx, b, d, beta, rho, iters, every):
            lib = load()
            _need(b, "b")
            d = d.detach().contiguous()
            _need(d, "d")
            shape = _shape_of(b, d)
            N, K = b.shape[0], d.shape[0]
            rho_t = _rho_tensor(rho, N, b.device)
            nck = (int(iters) + int(every) - 1) // int(every)
            z = torch.empty((N, K) + tuple(b.shape[2:]), dtype=torch.float32, device=b.device)
            rec = lib.csc_unrolled_record_floats(ctypes.byref(shape))
            ckpt = torch.empty(max(1, nck) * rec, dtype=torch.float32, device=b.device)
            ws, nbytes = _diff_ws(shape, every, b.device)
            _check(lib.csc_code_unrolled(ctypes.byref(shape), _ptr(b), _ptr(d), float(beta), _ptr(rho_t),
                                         int(iters), int(every), _ptr(z), _ptr(ckpt), ws, nbytes, _stream()))
            ctx.save_for_backward(b, d, rho_t, ckpt)
            ctx.cfg = (float(beta), int(iters), int(every))
            ctx.beta_is_tensor = isinstance(beta, torch.Tensor)
            return z

        @staticmethod
        def backward(ctx, zbar):
            lib = load()
            b, d, rho_t, ckpt = ctx.saved_tensors
            beta, iters, every = ctx.cfg
            shape = _shape_of(b, d)
            zbar = zbar.contiguous().to(torch.float32)
            dd = torch.empty_like(d)
            dbeta = torch.empty(1, dtype=torch.float64, device=b.device)
            ws, nbytes = _diff_ws(shape, every, b.device)
            _check(lib.csc_code_backward(ctypes.byref(shape), _ptr(b), _ptr(d), beta, _ptr(rho_t), iters, every,
                                         _ptr(ckpt), _ptr(zbar), _ptr(dd), _ptr(dbeta), ws, nbytes, _stream()))
            gb = dbeta.reshape(()) if ctx.beta_is_tensor else None
            return None, dd, gb, None, None, None

    class CSCLoss(torch.autograd.Function):
        """Objective of eq:CSC summed over images (float64 scalar), with
        gradients with respect to d, z and beta (csc_loss_grad)."""

        @staticmethod
        def forward(ctx, b, d, z, beta):
            lib = load()
            d = d.detach().contiguous()
            z = z.detach().contiguous()
            _need(b, "b")
            _need(d, "d")
            _need(z, "z")
            shape = _shape_of(b, d)
            loss = torch.empty(b.shape[0] + 1, dtype=torch.float64, device=b.device)
            zbar = torch.empty_like(z)
            dd = torch.empty_like(d)
            dbeta = torch.empty(1, dtype=torch.float64, device=b.device)
            ws, nbytes = _diff_ws(shape, 1, b.device)
            _check(lib.csc_loss_grad(ctypes.byref(shape), _ptr(b), _ptr(d), _ptr(z), float(beta), _ptr(loss),
                                     _ptr(zbar), _ptr(dd), _ptr(dbeta), ws, nbytes, _stream()))
            ctx.save_for_backward(zbar, dd, dbeta)
            ctx.beta_is_tensor = isinstance(beta, torch.Tensor)
            return loss[-1]

        @staticmethod
        def backward(ctx, g):
            zbar, dd, dbeta = ctx.saved_tensors
            gf = g.to(torch.float32)
            gb = (g * dbeta.reshape(())) if ctx.beta_is_tensor else None
            return None, dd * gf, zbar * gf, gb

    return CSCUnrolled, CSCLoss


_AUTOGRAD = None


def _autograd():
    global _AUTOGRAD
    if _AUTOGRAD is None:
        _AUTOGRAD = _make_unrolled()
    return _AUTOGRAD


def unrolled_code(b, d, beta, rho, iters: int, every: int = 5):
    """Codes after ``iters`` unrolled ADMM iterations from zero, differentiable
    in d and (when a tensor) beta; checkpoints every ``every`` iterations."""
    return _autograd()[0].apply(b, d, beta, rho, int(iters), int(every))


def csc_loss(b, d, z, beta):
    """Objective of eq:CSC (sum over images), differentiable in d, z, beta."""
    return _autograd()[1].apply(b, d, z, beta)
