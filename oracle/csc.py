"""FP64 oracle for dual-domain convolutional sparse coding (CSC).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU library or its binding.

Conventions (readings of the paper where it is loose; each is pinned by a test
against something other than this file):

* Arrays: images ``b`` [N][J][*grid]; filters ``d`` [K][J][*fsupp]; codes ``z``
  and the ADMM split variable ``theta`` [N][K][*grid].  ``grid`` is 2-D (H, W)
  or 3-D (T, H, W); all transforms act on the trailing ``len(grid)`` axes.
* DFT: unnormalised forward transform, inverse scaled by 1/D (numpy).
* Circular boundary conditions throughout (Sec. 3, the paper drops the
  boundary mask of Heide et al. and assumes circulant convolution matrices).
* Filter support: tap m of a filter sits at grid index m (corner anchored);
  S reads those indices back (the support projection of eq:Learning).
* Convolution (d * z)[p] = sum_m d[m] z[(p - m) mod grid]; its DFT is
  dhat * zhat with dhat = DFT(S^T d).  The transpose is correlation,
  conj(dhat) * . in the Fourier domain (D_k = F diag(dhat_k) F^H, Sec. 3.2).
* Higher-order (tensor) CSC, Sec. 3.3: channel j of image n is
  x_j = sum_k d_jk * z_k with the code maps z_k shared by all J channels.
* The sparsity weight is ``beta`` (eq:CSC); the coding dual variable is
  ``lam`` (eq:Inference_Dual); ``rho`` is the ADMM step (eq:Inference_solution).
"""
from __future__ import annotations

import numpy as np

_f64 = np.float64


def _axes(nd):
    return tuple(range(-nd, 0))


def _fft(x, nd):
    return np.fft.fftn(x, axes=_axes(nd))


def _ifft_real(x, nd):
    return np.real(np.fft.ifftn(x, axes=_axes(nd)))


def pad_filters(d, grid):
    """S^T: place the filter taps at grid indices [0, M) per axis (eq:Learning,
    the support projection S and its transpose).  d [..][*fsupp] -> [..][*grid]."""
    d = np.asarray(d, _f64)
    nd = len(grid)
    fs = d.shape[-nd:]
    out = np.zeros(d.shape[:-nd] + tuple(grid), _f64)
    out[(Ellipsis,) + tuple(slice(0, m) for m in fs)] = d
    return out


def crop(t, fsupp):
    """S: read the support indices [0, M) back (eq:Learning)."""
    nd = len(fsupp)
    return t[(Ellipsis,) + tuple(slice(0, m) for m in fsupp)]


def filter_spectra(d, grid):
    """dhat[j][k] = DFT(S^T d_kj) (Sec. 3.2, circulant diagonalisation).
    d [K][J][*fsupp] -> [J][K][*grid] complex128."""
    padded = pad_filters(d, grid)                      # [K][J][*grid]
    return np.swapaxes(_fft(padded, len(grid)), 0, 1)  # [J][K][*grid]


def reconstruct(d, z, grid=None):
    """D z: x_j = sum_k d_jk * z_k for every image (eq:CSC data term, Sec. 3.3
    for J > 1).  z [N][K][*grid] -> [N][J][*grid]."""
    z = np.asarray(z, _f64)
    nd = np.asarray(d).ndim - 2
    grid = z.shape[-nd:] if grid is None else grid
    dh = filter_spectra(d, grid)
    zh = _fft(z, nd)
    return _ifft_real(np.einsum("jk...,nk...->nj...", dh, zh), nd)


def nuclear_norm(z):
    """Sum of the singular values of every code map taken as an H x W matrix
    (the trailing two axes).  z [..][H][W] -> [..]."""
    return np.linalg.svd(np.asarray(z, _f64), compute_uv=False).sum(axis=-1)


def regularizer(z, reg="l1"):
    """The sparsity term per image without its weight: sum_k ||z_k||_1
    (eq:CSC), or with reg="nuclear" sum_k ||z_k||_* (the nuclear norm of
    each 2-D map, the low-rank regulariser of Sec. 5).  z [N][K][..] -> [N]."""
    z = np.asarray(z, _f64)
    if reg == "l1":
        return np.abs(z).sum(axis=tuple(range(1, z.ndim)))
    if reg == "nuclear":
        return nuclear_norm(z).sum(axis=1)
    raise ValueError(reg)


def objective(b, d, z, beta, reg="l1"):
    """eq:CSC: 1/2 ||x - sum_k d_k * z_k||^2 + beta sum_k ||z_k||_1, summed
    over channels (with reg="nuclear" the l1 norm becomes the nuclear norm of
    each map); returns (per-image values [N], total)."""
    b = np.asarray(b, _f64)
    z = np.asarray(z, _f64)
    res = b - reconstruct(d, z)
    red = tuple(range(1, b.ndim))
    per = 0.5 * (res * res).sum(axis=red) + beta * regularizer(z, reg)
    return per, float(per.sum())


def soft(u, t):
    """Soft threshold sign(u) max(|u| - t, 0)."""
    return np.sign(u) * np.maximum(np.abs(u) - t, 0.0)


def project_spectral_ball(u, beta):
    """Projection onto {theta : ||theta_k||_2 <= beta for every map}, the
    unit ball of the spectral norm (the dual norm of the nuclear norm) scaled
    by beta: with u_k = U diag(s) V^T, the projection is U diag(min(s, beta))
    V^T, map by map over the trailing two axes."""
    U, sv, Vt = np.linalg.svd(np.asarray(u, _f64), full_matrices=False)
    return (U * np.minimum(sv, beta)[..., None, :]) @ Vt


def svt(u, t):
    """Singular value thresholding U diag(max(s - t, 0)) V^T per map: the
    proximal operator of t ||.||_* (the nuclear-norm analogue of soft)."""
    U, sv, Vt = np.linalg.svd(np.asarray(u, _f64), full_matrices=False)
    return (U * np.maximum(sv - t, 0.0)[..., None, :]) @ Vt


def project_dual_ball(u, beta, reg="l1"):
    """Pi_C of eq:Inference_solution: C is the beta-ball of the dual norm of
    the regulariser: the l-infinity ball for l1 (a clip), the spectral-norm
    ball for the nuclear norm."""
    if reg == "l1":
        return np.clip(u, -beta, beta)
    if reg == "nuclear":
        return project_spectral_ball(u, beta)
    raise ValueError(reg)


def _gram(dh):
    """G_f = sum_k dhat_.k(f) dhat_.k(f)^H, a J x J Hermitian matrix per
    frequency: the Fourier diagonal of D D^T (Sec. 3.2; block-diagonal with
    D blocks of J x J for the tensor case, Sec. 3.3).  -> [*grid][J][J]."""
    return np.einsum("jk...,lk...->...jl", dh, np.conj(dh))


def _dual_solve(G, rhs, rho):
    """lambda-hat(f) = (G_f + I/rho)^-1 rhs(f), per image and frequency.
    G [*grid][J][J]; rhs [N][J][*grid]; rho [N]."""
    N, J = rhs.shape[:2]
    nd = rhs.ndim - 2
    r = np.moveaxis(rhs, 1, -1)                                  # [N][*grid][J]
    inv_rho = (1.0 / rho).reshape((N,) + (1,) * nd)
    if J == 1:
        lam = r[..., 0] / (G[None, ..., 0, 0].real + inv_rho)
        return lam[:, None]
    A = G[None] + inv_rho[..., None, None] * np.eye(J)
    lam = np.linalg.solve(A, r[..., None])[..., 0]
    return np.moveaxis(lam, -1, 1)


def _adapt_rho(rho, r_pri, r_dual, mu_b, tau_b):
    """Residual balancing (Boyd et al. 2011, Sec. 3.4.1; the paper cites that
    text for its ADMM updates).  z is the unscaled multiplier, so no rescale."""
    up = r_pri > mu_b * r_dual
    down = r_dual > mu_b * r_pri
    return np.where(up, rho * tau_b, np.where(down, rho / tau_b, rho))


def code(b, d, beta, rho, iters, z0=None, theta0=None, adaptive=False,
         rho_schedule=None, mu_b=10.0, tau_b=2.0, tol=None, reg="l1"):
    """Coding subproblem by ADMM on its dual (eq:Inference_Dual,
    eq:Inference_ADMM), literal updates of eq:Inference_solution in the
    Fourier domain, run for a fixed number of iterations per image (the coding
    problem separates over images, Sec. 3.1):

        lam   = (D D^T + I/rho)^-1 (D theta + D z / rho - x / rho)
        theta = Pi_C(D^T lam - z / rho),   C = {||theta||_inf <= beta}
        z     = z + rho (theta - D^T lam)

    Residuals per image (Boyd et al. 2011, Sec. 3.3, for the constraint
    theta = D^T lam): r_pri = ||theta' - D^T lam'||, r_dual = rho ||D (theta' - theta)||.

    rho: scalar or [N] (initial value).  ``rho_schedule`` [iters+1][N], if
    given, replaces the step used at each iteration (to replay a schedule).
    ``tol`` (convergence-driven mode): stop after the first iteration at which
    every image has r_pri <= tol sqrt(K D) and r_dual <= tol sqrt(J D), i.e.
    both RMS residuals at most tol (Boyd et al. 2011, Sec. 3.3.1, with zero
    relative tolerance); ``iters`` is then the largest count.
    ``reg="nuclear"`` replaces the l1 term by beta sum_k ||z_k||_* (Sec. 5:
    low-rank maps); C is then the spectral-norm ball (2-D grids only).
    Returns dict(z, theta, resid [done][N][2], rho [done+1][N], iters = done).
    """
    b = np.asarray(b, _f64)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    if reg == "nuclear" and nd != 2:
        raise ValueError("the nuclear norm is defined on 2-D maps")
    d = np.asarray(d, _f64)
    K = d.shape[0]
    dh = filter_spectra(d, grid)                     # [J][K][*grid]
    xh = _fft(b, nd)                                 # [N][J][*grid]
    G = _gram(dh)
    z = np.zeros((N, K) + grid) if z0 is None else np.array(z0, _f64)
    th = np.zeros((N, K) + grid) if theta0 is None else np.array(theta0, _f64)
    rho_v = np.broadcast_to(np.asarray(rho, _f64), (N,)).copy()
    if rho_schedule is not None:
        rho_schedule = np.asarray(rho_schedule, _f64)
        rho_v = rho_schedule[0].copy()
    sched = [rho_v.copy()]
    resid = []
    bshape = (N,) + (1,) * (nd + 1)
    for i in range(iters):
        r = rho_v.reshape(bshape)
        wh = _fft(th + z / r, nd)                                    # DFT(theta + z/rho)
        rhs = np.einsum("jk...,nk...->nj...", dh, wh) - xh / r       # D theta + D z/rho - x/rho
        lam = _dual_solve(G, rhs, rho_v)                             # [N][J][*grid]
        v = _ifft_real(np.einsum("jk...,nj...->nk...", np.conj(dh), lam), nd)  # D^T lam
        th_new = project_dual_ball(v - z / r, beta, reg)              # projection onto C
        z_new = z + r * (th_new - v)
        red = tuple(range(1, z.ndim))
        r_pri = np.sqrt(((th_new - v) ** 2).sum(axis=red))
        dth = _ifft_real(np.einsum("jk...,nk...->nj...", dh, _fft(th_new - th, nd)), nd)
        r_dual = rho_v * np.sqrt((dth ** 2).sum(axis=tuple(range(1, dth.ndim))))
        resid.append(np.stack([r_pri, r_dual], axis=-1))
        if rho_schedule is not None:
            rho_v = rho_schedule[i + 1].copy()
        elif adaptive:
            rho_v = _adapt_rho(rho_v, r_pri, r_dual, mu_b, tau_b)
        sched.append(rho_v.copy())
        z, th = z_new, th_new
        if tol is not None:
            npix = float(np.prod(grid))
            if np.all(r_pri <= tol * np.sqrt(K * npix)) and np.all(r_dual <= tol * np.sqrt(J * npix)):
                break
    done = len(resid)
    return {"z": z, "theta": th,
            "resid": np.array(resid).reshape(done, N, 2),
            "rho": np.array(sched), "iters": done}


def code_implicit(b, d, beta, rho, iters, z0=None, theta0=None):
    """The same iterates as :func:`code` (fixed rho) with theta eliminated.

    From the z update, theta' = D^T lam' + (z' - z)/rho, hence
    DFT(D theta') = G lam' + (DFT(D z') - DFT(D z)) / rho.  Keeping
    yhat = DFT(D z) and Thhat = DFT(D theta) per image, one iteration is

        lam'   = (G + I/rho)^-1 (Thhat + yhat/rho - xhat/rho)
        z'     = soft(z - rho D^T lam', rho beta)
        yhat'  = DFT(D z')
        Thhat' = G lam' + (yhat' - yhat)/rho

    and theta' = D^T lam' + (z' - z)/rho.  The z step is the Moreau
    decomposition of eq:Inference_solution's theta/z pair:
    z + rho (clip(v - z/rho, +-beta) - v) = soft(z - rho v, rho beta).
    """
    b = np.asarray(b, _f64)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    d = np.asarray(d, _f64)
    K = d.shape[0]
    dh = filter_spectra(d, grid)
    xh = _fft(b, nd)
    G = _gram(dh)
    z = np.zeros((N, K) + grid) if z0 is None else np.array(z0, _f64)
    th = np.zeros((N, K) + grid) if theta0 is None else np.array(theta0, _f64)
    rho_v = np.broadcast_to(np.asarray(rho, _f64), (N,)).copy()
    r = rho_v.reshape((N,) + (1,) * (nd + 1))
    yh = np.einsum("jk...,nk...->nj...", dh, _fft(z, nd))
    Th = np.einsum("jk...,nk...->nj...", dh, _fft(th, nd))
    theta = th
    for _ in range(iters):
        lam = _dual_solve(G, Th + (yh - xh) / r, rho_v)
        v = _ifft_real(np.einsum("jk...,nj...->nk...", np.conj(dh), lam), nd)
        z_new = soft(z - r * v, r * beta)
        yh_new = np.einsum("jk...,nk...->nj...", dh, _fft(z_new, nd))
        Glam = np.einsum("...jl,nl...->nj...", G, lam)
        Th = Glam + (yh_new - yh) / r
        theta = v + (z_new - z) / r
        z, yh = z_new, yh_new
    return {"z": z, "theta": theta}


def _cg(apply_a, rhs, x0, iters, tol=None):
    """Conjugate gradient (Hestenes-Stiefel) for the SPD system of
    eq:Learning_gamma, one independent system per channel (rhs and x0 are
    lists over channels, all stepped together), warm-started at x0, for
    ``iters`` iterations.  A zero residual or zero curvature stops the updates
    of that channel (step 0).  With ``tol`` the solve ends before any step
    once every channel has ||r_j|| <= tol ||rhs_j||.  Returns (x, steps)."""
    J = len(rhs)
    x = [x0[j].copy() for j in range(J)]
    r = [rhs[j] - apply_a(x[j]) for j in range(J)]
    p = [r[j].copy() for j in range(J)]
    rr = [float((r[j] * r[j]).sum()) for j in range(J)]
    bb = [float((rhs[j] * rhs[j]).sum()) for j in range(J)]

    def converged():
        return tol is not None and all(rr[j] <= tol * tol * bb[j] for j in range(J))

    steps = 0
    for _ in range(iters):
        if converged():
            break
        for j in range(J):
            ap = apply_a(p[j])
            pap = float((p[j] * ap).sum())
            alpha = rr[j] / pap if pap > 0 else 0.0
            x[j] = x[j] + alpha * p[j]
            r[j] = r[j] - alpha * ap
            rr_new = float((r[j] * r[j]).sum())
            beta_cg = rr_new / rr[j] if rr[j] > 0 else 0.0
            p[j] = r[j] + beta_cg * p[j]
            rr[j] = rr_new
        steps += 1
    return x, steps


def learn(b, z, fsupp, mu, gamma=None, inner_iters=10, cg_iters=10, cg_tol=None, info=None):
    """Learning subproblem in the dual (eq:Learning_Dual .. eq:mu_update).

    For fixed multipliers mu, gamma solves (eq:Learning_gamma)
        (I + sum_k 1/(2 mu_k) Z_k S^T S Z_k^T) gamma = -x
    by conjugate gradient with the convolutions applied in the Fourier domain
    and a warm start from the previous gamma; the filters follow from
    eq:Learning_Solution, d_k = -1/(2 mu_k) S Z_k^T gamma, and the multipliers
    from eq:mu_update, mu_k <- mu_k ||d_k||_2.  The images are coupled (all
    share the filters); Z_k^T p = sum_n Z_k^{n T} p^n.  For J > 1 the problem
    separates over channels (Sec. 3.3) with one operator and one gamma_j per
    channel; mu_k and the norm ||d_k|| span all channels.

    After the last multiplier update the filters are scaled into the unit
    ball, d_k / max(1, ||d_k||) (the constraint of eq:Learning).  A filter
    whose norm is exactly zero leaves its multiplier unchanged.  With
    ``cg_tol`` each CG solve ends once every channel's residual is at most
    cg_tol times its right-hand side (``cg_iters`` is then the largest count;
    it may also be a list with one count per multiplier update);
    ``info``, if a dict, receives the CG steps of each multiplier update
    under "cg_counts".
    Returns (d [K][J][*fsupp], mu [K], gamma [N][J][*grid]).
    """
    b = np.asarray(b, _f64)
    z = np.asarray(z, _f64)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    K = z.shape[1]
    zh = _fft(z, nd)                                              # [N][K][*grid]
    mu = np.array(np.broadcast_to(np.asarray(mu, _f64), (K,)))
    gamma = np.zeros_like(b) if gamma is None else np.array(gamma, _f64)
    kshape = (K,) + (1,) * nd

    def zt(p):            # sum_n Z_k^{n T} p^n  -> [K][*grid]
        return _ifft_real(np.einsum("nk...,n...->k...", np.conj(zh), _fft(p, nd)), nd)

    def zmul(u):          # Z_k^n u_k summed over k -> [N][*grid]
        return _ifft_real(np.einsum("nk...,k...->n...", zh, _fft(u, nd)), nd)

    def make_a(mu_):
        w = (1.0 / (2.0 * mu_)).reshape(kshape)

        def apply_a(p):
            return p + zmul(pad_filters(crop(zt(p), fsupp), grid) * w)
        return apply_a

    d = np.zeros((K, J) + tuple(fsupp))
    counts = []
    its = list(cg_iters) if np.ndim(cg_iters) else [cg_iters] * inner_iters
    for it in range(inner_iters):
        apply_a = make_a(mu)
        g, steps = _cg(apply_a, [-b[:, j] for j in range(J)], [gamma[:, j] for j in range(J)], its[it], cg_tol)
        counts.append(steps)
        for j in range(J):
            gamma[:, j] = g[j]
            d[:, j] = -crop(zt(gamma[:, j]), fsupp) / (2.0 * mu).reshape(kshape)
        nrm = np.sqrt((d.reshape(K, -1) ** 2).sum(axis=1))
        mu = np.where(nrm > 0, mu * nrm, mu)
    nrm = np.sqrt((d.reshape(K, -1) ** 2).sum(axis=1))
    d = d / np.maximum(1.0, nrm).reshape((K,) + (1,) * (d.ndim - 1))
    if isinstance(info, dict):
        info["cg_counts"] = counts
    return d, mu, gamma


def learn_dictionary(b, d0, beta, rho, t_in, t_out, inner_iters=10, cg_iters=10,
                     adaptive=False, tau=None, tol=None, cg_tol=None, reg="l1"):
    """Alg. 1 (coordinate descent between the two dual subproblems): z and
    theta start at zero and are carried (warm) into every later coding call,
    d starts from d0, mu at 1 and gamma at 0; each outer step codes, then
    learns.  Convergence-driven mode: ``tau`` ends the alternation after the
    first outer step whose objective (after learning) changed by at most tau
    relative to the previous step's (Sec. 4); ``tol`` and ``cg_tol`` are the
    stopping rules of code() and learn().  Returns dict(d, z, theta, mu,
    gamma, objectives, steps) where objectives lists f(d, z) after each half
    step and steps is the number of outer steps taken.  ``reg`` selects the
    regulariser of the coding step and the objective (see code)."""
    b = np.asarray(b, _f64)
    d = np.asarray(d0, _f64)
    N = b.shape[0]
    K = d.shape[0]
    fsupp = d.shape[2:]
    z = theta = None
    mu = np.ones(K)
    gamma = np.zeros_like(b)
    rho_v = np.broadcast_to(np.asarray(rho, _f64), (N,)).copy()
    objs = []
    steps = 0
    for _ in range(t_out):
        out = code(b, d, beta, rho_v, t_in, z, theta, adaptive=adaptive, tol=tol, reg=reg)
        z, theta = out["z"], out["theta"]
        if adaptive:
            rho_v = out["rho"][-1]
        objs.append(objective(b, d, z, beta, reg)[1])
        d, mu, gamma = learn(b, z, fsupp, mu, gamma, inner_iters, cg_iters, cg_tol)
        objs.append(objective(b, d, z, beta, reg)[1])
        steps += 1
        if tau is not None and len(objs) >= 4 and abs(objs[-1] - objs[-3]) <= tau * abs(objs[-3]):
            break
    return {"d": d, "z": z, "theta": theta, "mu": mu, "gamma": gamma,
            "objectives": objs, "steps": steps}


def objective_grad(b, d, z, beta):
    """Gradients of the objective of eq:CSC, f = sum_n 1/2 ||D z - x||^2 +
    beta ||z||_1: dz = D^T (D z - x) + beta sign(z) (sign(0) = 0),
    dd_jk[m] = sum_n sum_p (D z - x)_j[p] z_k[p - m], dbeta = ||z||_1.
    Returns (f, dz, dd, dbeta)."""
    b = np.asarray(b, _f64)
    z = np.asarray(z, _f64)
    d = np.asarray(d, _f64)
    nd = d.ndim - 2
    fsupp = d.shape[2:]
    grid = b.shape[2:]
    dh = filter_spectra(d, grid)
    res = reconstruct(d, z) - b
    f = 0.5 * (res ** 2).sum() + beta * np.abs(z).sum()
    dz = _ifft_real(np.einsum("jk...,nj...->nk...", np.conj(dh), _fft(res, nd)), nd) + beta * np.sign(z)
    dd = np.zeros(d.shape)
    for n in range(b.shape[0]):
        dd += _corr_crop(res[n], z[n], fsupp, nd)
    return float(f), dz, dd, float(np.abs(z).sum())


def _corr_crop(a, bsig, fsupp, nd):
    """c_jk[m] = sum_p a_j[p] b_k[p - m] for m in the support: the gradient of
    <a, d * b> with respect to the taps of d.  a [J][*grid], b [K][*grid] ->
    [K][J][*fsupp]."""
    ah = _fft(a, nd)
    bh = _fft(bsig, nd)
    c = _ifft_real(np.einsum("j...,k...->kj...", ah, np.conj(bh)), nd)
    return crop(c, fsupp)


def code_loss_grad(b, d, beta, rho, iters):
    """Loss and reference gradient of the unrolled coding solve.

    L(d, beta) = sum_n [1/2 ||x - D z^T||^2 + beta ||z^T||_1] where z^T is
    :func:`code` run ``iters`` times from z = theta = 0 at fixed rho.  The
    gradient is a hand-written reverse pass through every literal update of
    eq:Inference_solution (written with real operators:
    w = theta + z/rho, s = D w - x/rho, lam = P s with P = (D D^T + I/rho)^-1,
    v = D^T lam, u = v - z/rho, theta' = clip(u), z' = z + rho (theta' - v)),
    covering both places d enters: the iteration and the loss.  Kinks:
    clip passes the gradient iff |u| < beta strictly; d clip/d beta = sign(u)
    iff |u| > beta; d|z|/dz = sign(z) with sign(0) = 0.
    Returns (L, dL/dd [K][J][*fsupp], dL/dbeta).
    """
    b = np.asarray(b, _f64)
    d = np.asarray(d, _f64)
    N, J = b.shape[:2]
    grid = b.shape[2:]
    nd = len(grid)
    K = d.shape[0]
    fsupp = d.shape[2:]
    dh = filter_spectra(d, grid)
    G = _gram(dh)
    rho = float(rho)
    rho_n = np.full(N, rho)

    def Dop(w):           # [N][K] -> [N][J]
        return _ifft_real(np.einsum("jk...,nk...->nj...", dh, _fft(w, nd)), nd)

    def DTop(l):          # [N][J] -> [N][K]
        return _ifft_real(np.einsum("jk...,nj...->nk...", np.conj(dh), _fft(l, nd)), nd)

    def Pop(s):           # (D D^T + I/rho)^-1, symmetric
        return _ifft_real(_dual_solve(G, _fft(s, nd), rho_n), nd)

    z = np.zeros((N, K) + grid)
    th = np.zeros((N, K) + grid)
    tape = []
    for _ in range(iters):
        w = th + z / rho
        s = Dop(w) - b / rho
        lam = Pop(s)
        v = DTop(lam)
        u = v - z / rho
        th_new = np.clip(u, -beta, beta)
        z_new = z + rho * (th_new - v)
        tape.append((w, s, lam, v, u))
        z, th = z_new, th_new

    res = Dop(z) - b
    loss = 0.5 * (res ** 2).sum() + beta * np.abs(z).sum()
    gd = np.zeros((K, J) + tuple(fsupp))
    gbeta = np.abs(z).sum()
    for n in range(N):
        gd += _corr_crop(res[n], z[n], fsupp, nd)
    zbar = DTop(res) + beta * np.sign(z)
    thbar = np.zeros_like(zbar)
    for (w, s, lam, v, u) in reversed(tape):
        # z' = z + rho theta' - rho v
        tbar_tot = thbar + rho * zbar
        vbar = -rho * zbar
        zbar_prev = zbar.copy()
        # theta' = clip(u)
        inside = np.abs(u) < beta
        outside = np.abs(u) > beta
        ubar = tbar_tot * inside
        gbeta += (tbar_tot * np.sign(u) * outside).sum()
        # u = v - z/rho
        vbar = vbar + ubar
        zbar_prev += -ubar / rho
        # v = D^T lam
        lbar = Dop(vbar)
        # lam = P s
        sbar = Pop(lbar)
        # s = D w - x/rho
        wbar = DTop(sbar)
        # d contributions: C(lam, vbar - wbar) + C(sbar, w - v)
        for n in range(N):
            gd += _corr_crop(lam[n], vbar[n] - wbar[n], fsupp, nd)
            gd += _corr_crop(sbar[n], w[n] - v[n], fsupp, nd)
        # w = theta + z/rho
        thbar = wbar
        zbar = zbar_prev + wbar / rho
    return float(loss), gd, float(gbeta)
