"""Float32 emulation of the oracle's algorithm (test infrastructure).

The oracle runs every step in float64.  This module runs the same literal
steps -- the ADMM updates of eq:Inference_solution and the learning steps of
eq:Learning_gamma, eq:Learning_Solution and eq:mu_update with a
conjugate-gradient solve -- with every array in float32 / complex64
(scipy.fft keeps single precision), CG and norm reductions in float64 as on
the GPU.  Its distance from the oracle is the rounding floor that float32
arithmetic alone puts on a result: the GPU's tolerances are tied to it by
tests/test_float32_floor.py.  It shares no code with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

F32, C64 = np.float32, np.complex64


def _axes(nd):
    return tuple(range(-nd, 0))


def _place(t, fsupp, grid, dtype=F32):
    out = np.zeros(t.shape[:-len(grid)] + tuple(grid), dtype)
    out[(Ellipsis,) + tuple(slice(0, m) for m in fsupp)] = t
    return out


def _crop(t, fsupp):
    return t[(Ellipsis,) + tuple(slice(0, m) for m in fsupp)]


def code(b, d, beta, rho, iters, z0=None, theta0=None):
    """eq:Inference_solution for ``iters`` iterations at a fixed rho, in
    float32 (the oracle's ``code`` with single-precision arrays)."""
    b = np.asarray(b, F32)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    ax = _axes(nd)
    d = np.asarray(d, F32)
    K = d.shape[0]
    dh = np.swapaxes(sfft.fftn(_place(d, d.shape[2:], grid), axes=ax), 0, 1).astype(C64)   # [J][K]
    xh = sfft.fftn(b, axes=ax).astype(C64)
    G = np.einsum("jk...,lk...->...jl", dh, np.conj(dh)).astype(C64)
    z = np.zeros((N, K) + grid, F32) if z0 is None else np.array(z0, F32)
    th = np.zeros((N, K) + grid, F32) if theta0 is None else np.array(theta0, F32)
    r = F32(rho)
    for _ in range(iters):
        wh = sfft.fftn(th + z / r, axes=ax)
        rhs = np.einsum("jk...,nk...->nj...", dh, wh) - xh / r
        if J == 1:
            lam = rhs / (G[..., 0, 0].real + 1 / r)
        else:
            A = G[None] + (1 / r) * np.eye(J, dtype=C64)
            lam = np.moveaxis(np.linalg.solve(A, np.moveaxis(rhs, 1, -1)[..., None])[..., 0], -1, 1)
        v = sfft.ifftn(np.einsum("jk...,nj...->nk...", np.conj(dh), lam), axes=ax).real.astype(F32)
        th_new = np.clip(v - z / r, -beta, beta).astype(F32)
        z = (z + r * (th_new - v)).astype(F32)
        th = th_new
    return z, th


def learn(b, z, fsupp, mu, gamma, inner_iters, cg_iters):
    """The oracle's ``learn`` (fixed counts) with float32 arrays; CG scalars
    and filter norms are accumulated in float64."""
    b = np.asarray(b, F32)
    z = np.asarray(z, F32)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    ax = _axes(nd)
    K = z.shape[1]
    zh = sfft.fftn(z, axes=ax).astype(C64)
    mu = np.array(np.broadcast_to(np.asarray(mu, F32), (K,)))
    gamma = np.zeros_like(b) if gamma is None else np.array(gamma, F32)
    kshape = (K,) + (1,) * nd

    def zt(p):
        return sfft.ifftn(np.einsum("nk...,n...->k...", np.conj(zh), sfft.fftn(p, axes=ax)), axes=ax).real.astype(F32)

    def zmul(u):
        return sfft.ifftn(np.einsum("nk...,k...->n...", zh, sfft.fftn(u, axes=ax)), axes=ax).real.astype(F32)

    def dot(a, c):
        return float((a.astype(np.float64) * c).sum())

    d = np.zeros((K, J) + tuple(fsupp), F32)
    for _ in range(inner_iters):
        w = (1.0 / (2.0 * mu)).astype(F32).reshape(kshape)

        def apply_a(p):
            return p + zmul(_place(_crop(zt(p), fsupp), fsupp, grid) * w)

        for j in range(J):
            x = gamma[:, j].copy()
            r = (-b[:, j] - apply_a(x)).astype(F32)
            p = r.copy()
            rr = dot(r, r)
            for _ in range(cg_iters):
                ap = apply_a(p)
                pap = dot(p, ap)
                alpha = F32(rr / pap if pap > 0 else 0.0)
                x = (x + alpha * p).astype(F32)
                r = (r - alpha * ap).astype(F32)
                rr_new = dot(r, r)
                p = (r + F32(rr_new / rr if rr > 0 else 0.0) * p).astype(F32)
                rr = rr_new
            gamma[:, j] = x
            d[:, j] = -_crop(zt(x), fsupp) * w
        nrm = np.sqrt((d.reshape(K, -1).astype(np.float64) ** 2).sum(axis=1))
        mu = np.where(nrm > 0, mu * nrm, mu).astype(F32)
    nrm = np.sqrt((d.reshape(K, -1).astype(np.float64) ** 2).sum(axis=1))
    d = (d / np.maximum(1.0, nrm).reshape((K,) + (1,) * (d.ndim - 1))).astype(F32)
    return d, mu, gamma


def learn_dictionary(b, d0, beta, rho, t_in, t_out, inner_iters, cg_iters):
    """Alg. 1 (fixed rho and counts) in float32, state carried as in the
    oracle's ``learn_dictionary``.  Returns (d, z, mu, [(z, d) after each
    half step])."""
    d = np.asarray(d0, F32)
    z = th = gamma = None
    mu = np.ones(d.shape[0], F32)
    states = []
    for _ in range(t_out):
        z, th = code(b, d, beta, rho, t_in, z, th)
        states.append((z, d))
        d, mu, gamma = learn(b, z, d.shape[2:], mu, gamma, inner_iters, cg_iters)
        states.append((z, d))
    return d, z, mu, states


def code_loss_grad(b, d, beta, rho, iters):
    """The oracle's ``code_loss_grad`` (the unrolled coding solve from zero
    and its hand-written reverse pass) with every array in float32 /
    complex64; the loss and the beta gradient are summed in float64."""
    b = np.asarray(b, F32)
    d = np.asarray(d, F32)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    ax = _axes(nd)
    K = d.shape[0]
    fsupp = d.shape[2:]
    dh = np.swapaxes(sfft.fftn(_place(d, fsupp, grid), axes=ax), 0, 1).astype(C64)   # [J][K]
    G = np.einsum("jk...,lk...->...jl", dh, np.conj(dh)).astype(C64)
    r = F32(rho)

    def Dop(w):
        return sfft.ifftn(np.einsum("jk...,nk...->nj...", dh, sfft.fftn(w, axes=ax)), axes=ax).real.astype(F32)

    def DTop(l):
        return sfft.ifftn(np.einsum("jk...,nj...->nk...", np.conj(dh), sfft.fftn(l, axes=ax)), axes=ax).real.astype(F32)

    def Pop(s):
        sh = sfft.fftn(s, axes=ax)
        if J == 1:
            out = sh / (G[..., 0, 0].real + 1 / r)
        else:
            A = G[None] + (1 / r) * np.eye(J, dtype=C64)
            out = np.moveaxis(np.linalg.solve(A, np.moveaxis(sh, 1, -1)[..., None])[..., 0], -1, 1)
        return sfft.ifftn(out, axes=ax).real.astype(F32)

    def corr_crop(a, bsig):
        c = sfft.ifftn(np.einsum("j...,k...->kj...", sfft.fftn(a, axes=ax), np.conj(sfft.fftn(bsig, axes=ax))),
                       axes=ax).real.astype(F32)
        return _crop(c, fsupp)

    z = np.zeros((N, K) + grid, F32)
    th = np.zeros((N, K) + grid, F32)
    tape = []
    for _ in range(iters):
        w = (th + z / r).astype(F32)
        s = (Dop(w) - b / r).astype(F32)
        lam = Pop(s)
        v = DTop(lam)
        u = (v - z / r).astype(F32)
        th_new = np.clip(u, -beta, beta).astype(F32)
        z_new = (z + r * (th_new - v)).astype(F32)
        tape.append((w, s, lam, v, u))
        z, th = z_new, th_new
    res = Dop(z) - b
    loss = 0.5 * float((res.astype(np.float64) ** 2).sum()) + beta * float(np.abs(z.astype(np.float64)).sum())
    gd = np.zeros((K, J) + tuple(fsupp), F32)
    gbeta = float(np.abs(z.astype(np.float64)).sum())
    for n in range(N):
        gd += corr_crop(res[n], z[n])
    zbar = (DTop(res) + beta * np.sign(z)).astype(F32)
    thbar = np.zeros_like(zbar)
    for (w, s, lam, v, u) in reversed(tape):
        tbar_tot = (thbar + r * zbar).astype(F32)
        vbar = (-r * zbar).astype(F32)
        zbar_prev = zbar.copy()
        inside = np.abs(u) < beta
        outside = np.abs(u) > beta
        ubar = (tbar_tot * inside).astype(F32)
        gbeta += float((tbar_tot.astype(np.float64) * np.sign(u) * outside).sum())
        vbar = (vbar + ubar).astype(F32)
        zbar_prev = (zbar_prev - ubar / r).astype(F32)
        lbar = Dop(vbar)
        sbar = Pop(lbar)
        wbar = DTop(sbar)
        for n in range(N):
            gd += corr_crop(lam[n], vbar[n] - wbar[n])
            gd += corr_crop(sbar[n], w[n] - v[n])
        thbar = wbar
        zbar = (zbar_prev + wbar / r).astype(F32)
    return loss, gd.astype(np.float64), gbeta
