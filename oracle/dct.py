"""FP64 oracle of the DCT-domain variant (symmetric boundaries).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU legs,
never by the GPU library or its binding.

Sec. 3 notes (after Bristow et al.) that where the circular boundary of the
Fourier formulation is a problem the discrete cosine transform can take the
DFT's place.  Reading used here (the paper gives no formulas for it):

* Boundary: every image and code map is extended half-sample symmetrically
  about both ends of each axis (x[-1 - n] = x[n], x[2N - 1 - n] = x[n]), the
  extension the type-II DCT implies.
* Filters are whole-sample symmetric about their centre in each axis,
  h[m1, m2] = h[-m1, m2] = h[m1, -m2], and are given by one quadrant
  q [K][J][M1][M2]: h[m1, m2] = q[|m1|, |m2|] for |m1| < M1, |m2| < M2 (a
  (2 M1 - 1) x (2 M2 - 1) filter).  With both the extension and the filter
  symmetric, convolution of a map with h keeps the extension symmetric and
  the 2-D DCT-II diagonalises it with real eigenvalues
      hhat[k1, k2] = sum_{m1, m2} a(m1) a(m2) q[m1, m2] cos(pi k1 m1 / H) cos(pi k2 m2 / W),
  a(0) = 1, a(m > 0) = 2.  The operator is symmetric (D_k^T = D_k).
* Every update of eq:Inference_solution is then the paper's with the
  orthonormal 2-D DCT-II C in place of the DFT: D = C^T diag(hhat) C,
  D D^T is diagonal (J = 1) or block diagonal with real symmetric J x J
  blocks G_f = sum_k hhat_.k hhat_.k^T (J > 1), and no conjugates appear.

scipy's DCT (scipy.fft.dctn / idctn, type 2, orthonormal) is the library
primitive.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .csc import project_dual_ball, _adapt_rho

_f64 = np.float64


def dct2(x):
    """Orthonormal 2-D DCT-II over the last two axes."""
    return sfft.dctn(np.asarray(x, _f64), type=2, norm="ortho", axes=(-2, -1))


def idct2(x):
    """Inverse of dct2."""
    return sfft.idctn(np.asarray(x, _f64), type=2, norm="ortho", axes=(-2, -1))


def full_filter(q):
    """The whole-sample symmetric filter of quadrant q: [..][M1][M2] ->
    [..][2 M1 - 1][2 M2 - 1], centre at index (M1 - 1, M2 - 1)."""
    q = np.asarray(q, _f64)
    a = np.concatenate([q[..., :0:-1, :], q], axis=-2)
    return np.concatenate([a[..., :, :0:-1], a], axis=-1)


def eigenvalues(q, grid):
    """hhat[j][k] on the H x W grid of DCT frequencies, q [K][J][M1][M2] ->
    [J][K][H][W] (real)."""
    q = np.asarray(q, _f64)
    H, W = grid
    M1, M2 = q.shape[-2:]
    a1 = np.where(np.arange(M1) == 0, 1.0, 2.0)
    a2 = np.where(np.arange(M2) == 0, 1.0, 2.0)
    c1 = np.cos(np.pi * np.outer(np.arange(H), np.arange(M1)) / H) * a1     # [H][M1]
    c2 = np.cos(np.pi * np.outer(np.arange(W), np.arange(M2)) / W) * a2     # [W][M2]
    hh = np.einsum("am,kjmn,bn->jkab", c1, q, c2)
    return hh


def reconstruct(q, z):
    """D z for every image: x_j = sum_k h_jk *_s z_k, z [N][K][H][W] ->
    [N][J][H][W]."""
    z = np.asarray(z, _f64)
    hh = eigenvalues(q, z.shape[-2:])
    return idct2(np.einsum("jk...,nk...->nj...", hh, dct2(z)))


def objective(b, q, z, beta):
    """1/2 ||x - sum_k h_k *_s z_k||^2 + beta sum_k ||z_k||_1 (eq:CSC with the
    symmetric boundary); returns (per-image values [N], total)."""
    b = np.asarray(b, _f64)
    z = np.asarray(z, _f64)
    res = b - reconstruct(q, z)
    per = 0.5 * (res * res).sum(axis=(1, 2, 3)) + beta * np.abs(z).sum(axis=(1, 2, 3))
    return per, float(per.sum())


def _solve(G, rhs, rho):
    """lam(f) = (G_f + I/rho)^-1 rhs(f), real; G [H][W][J][J], rhs [N][J][H][W]."""
    N, J = rhs.shape[:2]
    inv_rho = (1.0 / rho).reshape(N, 1, 1)
    if J == 1:
        return (rhs[:, 0] / (G[None, ..., 0, 0] + inv_rho))[:, None]
    A = G[None] + inv_rho[..., None, None] * np.eye(J)
    r = np.moveaxis(rhs, 1, -1)[..., None]
    return np.moveaxis(np.linalg.solve(A, r)[..., 0], -1, 1)


def code(b, q, beta, rho, iters, z0=None, theta0=None, adaptive=False, rho_schedule=None, mu_b=10.0, tau_b=2.0):
    """Coding with symmetric boundaries: the literal updates of
    eq:Inference_solution with the DCT in place of the DFT,

        lam   = (D D^T + I/rho)^-1 (D theta + D z / rho - x / rho)
        theta = clip(D^T lam - z / rho, +-beta)
        z     = z + rho (theta - D^T lam),

    per image, for ``iters`` iterations; residuals and adaptive rho as in the
    circular oracle's code().  Returns dict(z, theta, resid [iters][N][2],
    rho [iters + 1][N])."""
    b = np.asarray(b, _f64)
    N, J, H, W = b.shape
    q = np.asarray(q, _f64)
    K = q.shape[0]
    hh = eigenvalues(q, (H, W))                        # [J][K][H][W]
    G = np.einsum("jkab,lkab->abjl", hh, hh)           # [H][W][J][J]
    xh = dct2(b)
    z = np.zeros((N, K, H, W)) if z0 is None else np.array(z0, _f64)
    th = np.zeros((N, K, H, W)) if theta0 is None else np.array(theta0, _f64)
    rho_v = np.broadcast_to(np.asarray(rho, _f64), (N,)).copy()
    if rho_schedule is not None:
        rho_schedule = np.asarray(rho_schedule, _f64)
        rho_v = rho_schedule[0].copy()
    sched = [rho_v.copy()]
    resid = []
    for i in range(iters):
        r = rho_v.reshape(N, 1, 1, 1)
        wh = dct2(th + z / r)
        rhs = np.einsum("jkab,nkab->njab", hh, wh) - xh / r
        lam = _solve(G, rhs, rho_v)
        v = idct2(np.einsum("jkab,njab->nkab", hh, lam))
        th_new = project_dual_ball(v - z / r, beta)
        z_new = z + r * (th_new - v)
        r_pri = np.sqrt(((th_new - v) ** 2).sum(axis=(1, 2, 3)))
        dth = np.einsum("jkab,nkab->njab", hh, dct2(th_new - th))
        r_dual = rho_v * np.sqrt((dth ** 2).sum(axis=(1, 2, 3)))
        resid.append(np.stack([r_pri, r_dual], axis=-1))
        if rho_schedule is not None:
            rho_v = rho_schedule[i + 1].copy()
        elif adaptive:
            rho_v = _adapt_rho(rho_v, r_pri, r_dual, mu_b, tau_b)
        sched.append(rho_v.copy())
        z, th = z_new, th_new
    return {"z": z, "theta": th, "resid": np.array(resid).reshape(len(resid), N, 2), "rho": np.array(sched)}
