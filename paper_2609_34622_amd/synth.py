"""Seeded synthetic inputs for the BMND workloads.

This module holds no part of the denoising arithmetic: it only draws clean
means and Poisson counts.  The observation model is the paper's scaled
Poisson model in processing units (section Experiments, Noise Models):
``K ~ Poi(lambda)``, ``y = s_P K`` with ``s_P = 1 / lambda_pk``.  Arrays are
float32, C-order.  Every generator is a pure function of its seed
(``numpy.random.Generator(PCG64(seed))``).

Workloads (stand-ins for the paper's datasets, which are not available):
  * ``image_2d_small``  — 128x128 piecewise-constant discs/rectangles +
    gradient + sinusoidal texture, peak 30 counts;
  * ``ecg_batch``       — quasi-periodic ECG-like signals at 500 Hz, baseline
    5, peak 50 counts;
  * ``microscopy_2d``   — Gaussian blobs + random-walk filaments on
    background 2, peak log-uniform in [5, 100];
  * ``phantom_3d``      — nested ellipsoids + smooth background, low counts.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Sample:
    y: np.ndarray        # float32 observation, processing units (s_P * counts)
    x: np.ndarray        # float32 clean mean, same units
    s_p: float           # Poisson scale = 1 / lambda_pk
    lam_pk: float


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _observe(rng: np.random.Generator, lam: np.ndarray, lam_pk: float) -> Sample:
    lam = np.maximum(lam, 0.0)
    k = rng.poisson(lam).astype(np.float64)
    s_p = 1.0 / float(lam_pk)
    y = (k * s_p).astype(np.float32)
    x = (lam * s_p).astype(np.float32)
    return Sample(y=y, x=x, s_p=s_p, lam_pk=float(lam_pk))


def image_2d_small(seed: int = 1000, size: int = 128, peak: float = 30.0) -> Sample:
    """Discs and rectangles (levels U[0.2, 0.8], painted in order) over a
    0.25 linear gradient along (i + j), plus 0.1 sinusoidal texture of
    period U[6, 16] px in a random direction; clipped at 0, max scaled to 1,
    lambda = peak * x."""
    rng = _rng(seed)
    n = size
    ii, jj = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                         indexing="ij")
    img = 0.25 * (ii + jj) / (2.0 * (n - 1))
    for _ in range(6):
        r = rng.uniform(6, 24) * n / 128.0
        ci, cj = rng.uniform(0, n, size=2)
        lev = rng.uniform(0.2, 0.8)
        img[(ii - ci) ** 2 + (jj - cj) ** 2 <= r * r] = lev
    for _ in range(4):
        h, w = rng.uniform(8, 40, size=2) * n / 128.0
        ci, cj = rng.uniform(0, n, size=2)
        lev = rng.uniform(0.2, 0.8)
        img[(np.abs(ii - ci) <= h / 2) & (np.abs(jj - cj) <= w / 2)] = lev
    per = rng.uniform(6, 16)
    th = rng.uniform(0, np.pi)
    img = img + 0.1 * np.sin(2 * np.pi * (ii * np.cos(th) + jj * np.sin(th)) / per)
    img = np.clip(img, 0.0, None)
    img /= img.max()
    return _observe(rng, peak * img, peak)


def ecg_signal(rng: np.random.Generator, length: int, fs: float = 500.0) -> np.ndarray:
    """Sum of five Gaussian bumps (P, Q, R, S, T) per beat, RR = 0.8 s (+-10 %),
    amplitudes +-10 % per beat."""
    t = np.arange(length, dtype=np.float64) / fs
    sig = np.zeros(length)
    waves = [(-0.20, 0.025, 0.12), (-0.035, 0.010, -0.06), (0.0, 0.012, 1.0),
             (0.035, 0.010, -0.08), (0.28, 0.060, 0.30)]
    tr = rng.uniform(0.0, 0.8)
    while tr < t[-1] + 0.5:
        for off, wd, amp in waves:
            a = amp * rng.uniform(0.9, 1.1)
            c = tr + off
            lo = max(0, int((c - 5 * wd) * fs))
            hi = min(length, int((c + 5 * wd) * fs) + 1)
            if hi > lo:
                sig[lo:hi] += a * np.exp(-0.5 * ((t[lo:hi] - c) / wd) ** 2)
        tr += 0.8 * rng.uniform(0.9, 1.1)
    return sig


def ecg_batch(n_signals: int = 256, length: int = 65536, seed: int = 2000,
              baseline: float = 5.0, peak: float = 50.0) -> Sample:
    """Batch of ECG-like signals offset to `baseline` counts and scaled to
    `peak` counts: lambda = max(baseline + (peak - baseline) s / max s, 0)."""
    rng = _rng(seed)
    lam = np.empty((n_signals, length))
    for b in range(n_signals):
        s = ecg_signal(rng, length)
        smax = s.max()
        shape = s / smax if smax > 0 else np.zeros_like(s)  # no beat in very short signals
        lam[b] = np.maximum(baseline + (peak - baseline) * shape, 0.0)
    return _observe(rng, lam, peak)


def _stamp_gauss2d(img: np.ndarray, ci: float, cj: float, sig: float, amp: float):
    n0, n1 = img.shape
    r = int(np.ceil(4 * sig))
    i0, i1 = max(0, int(ci) - r), min(n0, int(ci) + r + 2)
    j0, j1 = max(0, int(cj) - r), min(n1, int(cj) + r + 2)
    if i1 <= i0 or j1 <= j0:
        return
    ii = np.arange(i0, i1)[:, None] - ci
    jj = np.arange(j0, j1)[None, :] - cj
    img[i0:i1, j0:j1] += amp * np.exp(-0.5 * (ii * ii + jj * jj) / (sig * sig))


def microscopy_2d(seed: int = 3000, size: int = 1024, background: float = 2.0) -> Sample:
    """U{200..2000} isotropic Gaussian blobs (sigma U[1, 6] px, amplitude
    U[0.2, 1]) plus U{5..30} random-walk filaments (200-1000 unit steps,
    heading noise N(0, 0.2 rad), cross-section sigma U[0.5, 1] px, amplitude
    U[0.3, 1]); f scaled to max 1; lambda = background + (peak - background) f
    with peak log-uniform in [5, 100]."""
    rng = _rng(seed)
    img = np.zeros((size, size))
    for _ in range(int(rng.integers(200, 2001))):
        ci, cj = rng.uniform(0, size, size=2)
        _stamp_gauss2d(img, ci, cj, rng.uniform(1, 6), rng.uniform(0.2, 1.0))
    for _ in range(int(rng.integers(5, 31))):
        ci, cj = rng.uniform(0, size, size=2)
        head = rng.uniform(0, 2 * np.pi)
        sig = rng.uniform(0.5, 1.0)
        amp = rng.uniform(0.3, 1.0)
        steps = int(rng.integers(200, 1001))
        fil = np.zeros_like(img)
        for _ in range(steps):
            head += rng.normal(0.0, 0.2)
            ci += np.cos(head)
            cj += np.sin(head)
            if not (0 <= ci < size and 0 <= cj < size):
                break
            _stamp_gauss2d(fil, ci, cj, sig, 1.0)
        if fil.max() > 0:
            img += amp * fil / fil.max()
    img /= img.max()
    peak = float(np.exp(rng.uniform(np.log(5.0), np.log(100.0))))
    lam = background + (peak - background) * img
    return _observe(rng, lam, peak)


def phantom_3d(seed: int = 4000, shape=(256, 256, 128)) -> Sample:
    """U{10..30} nested ellipsoids painted largest first (semi-axes
    U[10,100] x U[10,100] x U[5,50] voxels, random rotation, activity
    U[0.5, 10] counts) over a white-noise background smoothed by a Gaussian
    of sigma 8 voxels and rescaled to [0, 0.5]; lambda_pk = max lambda."""
    from scipy.ndimage import gaussian_filter

    rng = _rng(seed)
    bg = gaussian_filter(rng.standard_normal(shape), sigma=8.0, mode="wrap")
    bg = 0.5 * (bg - bg.min()) / (bg.max() - bg.min())
    lam = bg.copy()
    n_ell = int(rng.integers(10, 31))
    ells = []
    for _ in range(n_ell):
        ax = np.array([rng.uniform(10, 100), rng.uniform(10, 100), rng.uniform(5, 50)])
        ax *= np.array(shape) / np.array([256.0, 256.0, 128.0])
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                      [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                      [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        c = rng.uniform(0, 1, size=3) * np.array(shape)
        act = rng.uniform(0.5, 10.0)
        ells.append((np.prod(ax), ax, R, c, act))
    ells.sort(key=lambda e: -e[0])
    for _, ax, R, c, act in ells:
        r = int(np.ceil(ax.max()))
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, np.array(shape))
        if np.any(hi <= lo):
            continue
        g = np.stack(np.meshgrid(*[np.arange(lo[d], hi[d]) - c[d] for d in range(3)],
                                 indexing="ij"), axis=-1)
        loc = g @ R
        inside = ((loc / ax) ** 2).sum(-1) <= 1.0
        sub = lam[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub[inside] = act
    lam_pk = float(lam.max())
    return _observe(rng, lam, lam_pk)


@dataclass
class GaussianSample:
    y: np.ndarray        # float32 observation x + n
    x: np.ndarray        # float32 clean signal
    psd: np.ndarray      # float64 power spectral density of n on the array's DFT grid
    sigma: float         # marginal standard deviation of n


def correlated_gaussian(shape, seed: int = 8000, sigma: float = 0.1, corr_len=1.0) -> GaussianSample:
    """Clean signal (the 1-D ECG beats, the 2-D disc/rectangle scene, the
    3-D ellipsoid phantom, scaled to peak 1) plus stationary correlated
    Gaussian noise n = h (*) w: white unit noise w filtered circularly by a
    separable Gaussian kernel h of standard deviation ``corr_len`` samples
    per axis (truncated at 3 corr_len), scaled so that n has standard
    deviation ``sigma``.  Its spectral density samples are |Omega| |DFT(h)|^2
    (unnormalised DFT; a white field of variance s^2 has |Omega| s^2)."""
    shape = tuple(int(v) for v in shape)
    if len(shape) == 1:
        x = ecg_batch(n_signals=1, length=shape[0], seed=seed).x[0]
    elif len(shape) == 2:
        x = image_2d_small(seed, size=max(shape)).x[: shape[0], : shape[1]]
    else:
        x = phantom_3d(seed, shape=shape).x
    x = np.asarray(x, np.float64)
    x = x / max(float(x.max()), 1e-30)
    cl = np.broadcast_to(np.asarray(corr_len, np.float64), (len(shape),))
    h = np.ones((1,) * len(shape))
    for d, n in enumerate(shape):
        r = int(np.ceil(3 * cl[d])) if cl[d] > 0 else 0
        t = np.arange(-r, r + 1, dtype=np.float64)
        k = np.exp(-0.5 * (t / cl[d]) ** 2) if cl[d] > 0 else np.ones(1)
        kk = np.zeros(n)
        for v, tt in zip(k, t):
            kk[int(tt) % n] += v
        h = h * kk.reshape((1,) * d + (n,) + (1,) * (len(shape) - d - 1))
    h *= sigma / np.sqrt((h ** 2).sum())
    Hf = np.fft.fftn(h)
    rng = _rng(seed + 1)
    w = rng.normal(0.0, 1.0, shape)
    n = np.real(np.fft.ifftn(np.fft.fftn(w) * Hf))
    psd = float(np.prod(shape)) * np.abs(Hf) ** 2
    return GaussianSample(y=(x + n).astype(np.float32), x=x.astype(np.float32),
                          psd=np.ascontiguousarray(psd), sigma=float(sigma))
