"""Seeded synthetic inputs for dual-domain convolutional sparse coding.

This module is shared by the FP64 oracle's tests, the GPU parity tests and the
benchmark.  It holds none of the method's arithmetic: it only draws images and
initial filters with the shapes and statistics of the paper's workloads
(Sec. 4.1, "Implementation Details": grayscale and colour image sets, a colour
video; contrast-normalised inputs; randomly initialised filters).  The paper's
own datasets are not used; 1/f-spectrum Gaussian fields stand in for natural
images because natural images have an approximately 1/f amplitude spectrum.

Recipe (all in float64 from ``numpy.random.default_rng`` (PCG64), rounded once
to float32 at the end):

* 1/f field: white N(0,1) field -> DFT -> multiply by 1/max(|f|, 1/L) with |f|
  in cycles/sample and L the largest side, DC set to 0 -> real inverse DFT.
* colour: three independent 1/f fields mixed by the Cholesky factor of the
  channel correlation matrix [[1,.8,.8],[.8,1,.8],[.8,.8,1]].
* local contrast normalisation per channel (and per frame): Gaussian
  sigma = 2 px with circular boundary,  x <- x - G*x,  x <- x / sqrt(G*x^2 + 0.01),
  then zero mean and unit standard deviation per image, then times ``amp``.
* zero padding at the bottom/right edge up to the FFT grid.
* filters: i.i.d. N(0,1) taps scaled to unit L2 norm per filter (over all
  channels and taps).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "one_over_f",
    "contrast_normalize",
    "gray_images",
    "rgb_images",
    "rgb_video",
    "unit_filters",
    "ragged_sizes",
    "next_pow2",
    "CSCConfig",
    "CONFIGS",
    "make_inputs",
]


def next_pow2(n: int) -> int:
    return 1 << max(0, int(n - 1).bit_length())


def one_over_f(rng: np.random.Generator, shape: Sequence[int]) -> np.ndarray:
    """Gaussian field with a 1/|f| amplitude spectrum, float64."""
    shape = tuple(int(s) for s in shape)
    white = rng.standard_normal(shape)
    spec = np.fft.fftn(white)
    grids = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    fr = np.sqrt(sum(g * g for g in grids))
    big = max(shape)
    gain = 1.0 / np.maximum(fr, 1.0 / big)
    gain[(0,) * len(shape)] = 0.0
    return np.real(np.fft.ifftn(spec * gain))


def _gauss_blur_circular(x: np.ndarray, sigma: float) -> np.ndarray:
    """Separable circular Gaussian blur over the last two axes."""
    rad = int(math.ceil(3 * sigma))
    taps = np.exp(-0.5 * (np.arange(-rad, rad + 1) / sigma) ** 2)
    taps /= taps.sum()
    out = x
    for axis in (-2, -1):
        acc = np.zeros_like(out)
        for t, w in zip(range(-rad, rad + 1), taps):
            acc += w * np.roll(out, t, axis=axis)
        out = acc
    return out


def contrast_normalize(x: np.ndarray, sigma: float = 2.0) -> np.ndarray:
    """Local contrast normalisation over the last two axes, then global
    zero-mean / unit-std over the last two axes (and any leading channel or
    frame axes of a single image passed in)."""
    x = np.asarray(x, np.float64)
    x = x - _gauss_blur_circular(x, sigma)
    x = x / np.sqrt(_gauss_blur_circular(x * x, sigma) + 0.01)
    x = x - x.mean()
    sd = x.std()
    return x / sd if sd > 0 else x


def _pad_to(x: np.ndarray, grid: Sequence[int]) -> np.ndarray:
    out = np.zeros(x.shape[: x.ndim - len(grid)] + tuple(grid), x.dtype)
    sl = tuple(slice(0, s) for s in x.shape[x.ndim - len(grid):])
    out[(Ellipsis,) + sl] = x
    return out


def gray_images(n: int, size: Tuple[int, int], amp: float, seed: int,
                grid: Optional[Tuple[int, int]] = None) -> np.ndarray:
    """[n][1][H][W] float32 contrast-normalised 1/f images, zero-padded to grid."""
    rng = np.random.default_rng(seed)
    imgs = []
    for _ in range(n):
        f = contrast_normalize(one_over_f(rng, size)) * amp
        imgs.append(f[None])
    out = np.stack(imgs)
    if grid is not None and tuple(grid) != tuple(size):
        out = _pad_to(out, grid)
    return out.astype(np.float32)


_RGB_CORR = np.array([[1.0, 0.8, 0.8], [0.8, 1.0, 0.8], [0.8, 0.8, 1.0]])


def rgb_images(n: int, size: Tuple[int, int], amp: float, seed: int) -> np.ndarray:
    """[n][3][H][W] float32: three 1/f fields mixed to correlation 0.8, each
    channel contrast-normalised."""
    rng = np.random.default_rng(seed)
    chol = np.linalg.cholesky(_RGB_CORR)
    out = []
    for _ in range(n):
        raw = np.stack([one_over_f(rng, size) for _ in range(3)])
        raw /= raw.std(axis=(1, 2), keepdims=True)
        mixed = np.einsum("cd,dhw->chw", chol, raw)
        out.append(np.stack([contrast_normalize(c) * amp for c in mixed]))
    return np.stack(out).astype(np.float32)


def rgb_video(frames: int, size: Tuple[int, int], amp: float, seed: int) -> np.ndarray:
    """[1][3][T][H][W] float32: 3-D 1/f fields (spectrum over t, y, x) mixed to
    channel correlation 0.8; contrast normalisation per channel and frame."""
    rng = np.random.default_rng(seed)
    chol = np.linalg.cholesky(_RGB_CORR)
    shape = (frames,) + tuple(size)
    raw = np.stack([one_over_f(rng, shape) for _ in range(3)])
    raw /= raw.std(axis=(1, 2, 3), keepdims=True)
    mixed = np.einsum("cd,dthw->cthw", chol, raw)
    out = np.empty_like(mixed)
    for c in range(3):
        for t in range(frames):
            out[c, t] = contrast_normalize(mixed[c, t]) * amp
    return out[None].astype(np.float32)


def unit_filters(k: int, j: int, fsupp: Sequence[int], seed: int) -> np.ndarray:
    """[K][J][*fsupp] float32, i.i.d. N(0,1) taps with unit L2 norm per filter."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((k, j) + tuple(fsupp))
    nrm = np.sqrt((d.reshape(k, -1) ** 2).sum(axis=1))
    d /= nrm.reshape((k,) + (1,) * (d.ndim - 1))
    return d.astype(np.float32)


def symmetric_quadrants(k: int, j: int, m: Sequence[int], seed: int) -> np.ndarray:
    """[K][J][M1][M2] float32 quadrants of whole-sample symmetric filters
    (h[m1][m2] = q[|m1|][|m2|], (2 M1 - 1) x (2 M2 - 1) taps): i.i.d. N(0,1)
    quadrant taps, scaled so that each full filter has unit L2 norm (a tap
    off an axis appears four times, one on an axis twice, the centre once)."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((k, j) + tuple(m))
    mult = np.outer(np.where(np.arange(m[0]) == 0, 1.0, 2.0), np.where(np.arange(m[1]) == 0, 1.0, 2.0))
    nrm = np.sqrt((q ** 2 * mult).reshape(k, -1).sum(axis=1))
    q /= nrm.reshape(k, 1, 1, 1)
    return q.astype(np.float32)


def ragged_sizes(n: int, lo: int, hi: int, seed: int, square: bool = False):
    """List of n (H, W) sides drawn uniformly from {lo..hi} (independently per
    axis unless ``square``)."""
    rng = np.random.default_rng(seed)
    if square:
        s = rng.integers(lo, hi + 1, size=n)
        return [(int(a), int(a)) for a in s]
    hw = rng.integers(lo, hi + 1, size=(n, 2))
    return [(int(a), int(b)) for a, b in hw]


@dataclasses.dataclass(frozen=True)
class CSCConfig:
    """One synthetic workload.  ``beta`` is the sparsity weight of the CSC
    objective; ``rho`` the ADMM step (None = adaptive residual balancing
    started from ``rho0``)."""
    name: str
    index: int
    n: int
    j: int
    k: int
    size: Tuple[int, ...]          # image size before padding (2-D or 3-D)
    grid: Tuple[int, ...]          # FFT grid
    fsupp: Tuple[int, ...]
    beta: float
    rho: Optional[float]
    rho0: float
    t_in: int
    t_out: int
    amp: float
    kind: str = "gray"             # gray | rgb | video | ragged
    learn_inner: int = 10          # mu iterations per learning call
    learn_cg: int = 10             # CG iterations per gamma solve

    @property
    def image_seed(self) -> int:
        return 1000 + self.index

    @property
    def filter_seed(self) -> int:
        return 2000 + self.index


# Amplitudes were chosen so that oracle code densities after the configured
# iteration counts fall inside [1%, 30%]; unit-std inputs at rho=10 give
# all-zero codes for beta=1, which would make any comparison vacuous.
# Measured densities: small 5.4%, small_rho01 11.7%, learn 8.1% (2 images),
# tensor 6.0% (2 images), batched 1.1-1.9% (3 images), unrolled_fd 24.8%.
CONFIGS = {
    "small": CSCConfig("small", 0, n=4, j=1, k=16, size=(64, 64), grid=(64, 64),
                       fsupp=(11, 11), beta=1.0, rho=10.0, rho0=10.0, t_in=20,
                       t_out=2, amp=10.0),
    "small_rho01": CSCConfig("small_rho01", 0, n=4, j=1, k=16, size=(64, 64),
                             grid=(64, 64), fsupp=(11, 11), beta=1.0, rho=0.1,
                             rho0=0.1, t_in=20, t_out=2, amp=1.0),
    "learn": CSCConfig("learn", 1, n=10, j=1, k=100, size=(100, 100),
                       grid=(128, 128), fsupp=(11, 11), beta=1.0, rho=None,
                       rho0=10.0, t_in=10, t_out=20, amp=10.0),
    "tensor": CSCConfig("tensor", 2, n=32, j=3, k=64, size=(128, 128),
                        grid=(128, 128), fsupp=(11, 11), beta=0.5, rho=10.0,
                        rho0=10.0, t_in=20, t_out=10, amp=10.0, kind="rgb"),
    "video": CSCConfig("video", 2, n=1, j=3, k=64, size=(16, 128, 128),
                       grid=(16, 128, 128), fsupp=(3, 11, 11), beta=0.5,
                       rho=10.0, rho0=10.0, t_in=20, t_out=10, amp=10.0,
                       kind="video"),
    "batched": CSCConfig("batched", 3, n=256, j=1, k=64, size=(256, 256),
                         grid=(256, 256), fsupp=(11, 11), beta=1.0, rho=10.0,
                         rho0=10.0, t_in=30, t_out=1, amp=30.0, kind="ragged"),
    "unrolled": CSCConfig("unrolled", 4, n=16, j=1, k=100, size=(256, 256),
                          grid=(256, 256), fsupp=(11, 11), beta=1.0, rho=10.0,
                          rho0=10.0, t_in=30, t_out=1, amp=30.0),
    "unrolled_fd": CSCConfig("unrolled_fd", 4, n=2, j=1, k=4, size=(32, 32),
                             grid=(32, 32), fsupp=(11, 11), beta=1.0, rho=10.0,
                             rho0=10.0, t_in=30, t_out=1, amp=10.0),
}


def _vary(base: str, tag: str, **kw) -> CSCConfig:
    return dataclasses.replace(CONFIGS[base], name="%s_%s" % (base, tag), **kw)


# Scaling sweeps over the number of filters K and of images N (the shapes of
# the paper's scalability study, Sec. 5.3, and of its TCSC study on colour
# images and video, Sec. 5.4), on this generator: gray 100 x 100 images
# (128^2 grid) around the alternation workload; RGB 128^2 images at ten
# images or K = 64; the RGB video volume.  K = 49 and K = 100 are the paper's
# own dictionary sizes.  Each point keeps its base workload's seeds, steps
# and iteration counts (images are the first N of the base set where N is
# not larger).
SWEEPS = {
    "gray_K": [_vary("learn", "K%d" % k, k=k) for k in (16, 25, 36, 49, 64, 81, 100)],
    "gray_N": [_vary("learn", "N%d" % n, n=n) for n in (1, 2, 5, 10, 20, 50, 100)],
    "rgb_K": [_vary("tensor", "K%d" % k, n=10, k=k) for k in (8, 16, 32, 64, 100)],
    "rgb_N": [_vary("tensor", "N%d" % n, n=n) for n in (1, 5, 10, 20, 50, 100)],
    "video_K": [_vary("video", "K%d" % k, k=k) for k in (8, 16, 32, 64)],
}


def make_inputs(cfg: CSCConfig, n: Optional[int] = None):
    """(b, d0) for a uniform-grid config: b [N][J][*grid] f32, d0 [K][J][*fsupp] f32.
    ``n`` limits the number of images (the first n of the full set)."""
    nn = cfg.n if n is None else min(n, cfg.n)
    if cfg.kind == "gray":
        b = gray_images(cfg.n, cfg.size, cfg.amp, cfg.image_seed, cfg.grid)[:nn]
    elif cfg.kind == "rgb":
        b = rgb_images(cfg.n, cfg.size, cfg.amp, cfg.image_seed)[:nn]
    elif cfg.kind == "video":
        b = rgb_video(cfg.size[0], cfg.size[1:], cfg.amp, cfg.image_seed)
    else:
        raise ValueError("ragged configs use ragged_inputs()")
    d0 = unit_filters(cfg.k, cfg.j, cfg.fsupp, cfg.filter_seed)
    return np.ascontiguousarray(b), d0


def ragged_inputs(cfg: CSCConfig, n: Optional[int] = None, lo: int = 48,
                  hi: int = 256, square: bool = False):
    """List of per-image arrays [1][H][W] f32 (unpadded) plus their padded
    grids and the shared filters, for the batched workload."""
    nn = cfg.n if n is None else min(n, cfg.n)
    sizes = ragged_sizes(cfg.n, lo, hi, 3000, square)[:nn]
    rng = np.random.default_rng(cfg.image_seed)
    imgs, grids = [], []
    for (h, w) in sizes:
        f = contrast_normalize(one_over_f(rng, (h, w))) * cfg.amp
        imgs.append(f[None].astype(np.float32))
        grids.append((next_pow2(h), next_pow2(w)))
    d0 = unit_filters(cfg.k, cfg.j, cfg.fsupp, cfg.filter_seed)
    return imgs, grids, d0
