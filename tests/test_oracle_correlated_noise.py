"""Pins of the oracle's stationary correlated Gaussian noise model (section
Observation Models, Def. wide-sense stationary Gaussian noise; Prop. Gaussian
SSD noise bias; Lemma covariance propagation), independent of its formulas:

- the autocovariance from the power spectral density equals the closed form
  of noise made by circular filtering of white noise;
- Monte Carlo over such noise: the corrected SSD has mean zero for every
  candidate, and the empirical variance of every transformed coefficient of
  a group (overlapping members included) matches the propagated variance;
- a white spectrum reduces the model to white Gaussian noise with every
  plane exact (the full-covariance model treats repeated voxels exactly);
- the propagated variances equal the diagonal of an explicitly assembled
  Kronecker transform applied to an explicitly assembled group covariance.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def _kernel_psd(shape, h, sigma):
    """Noise n = h (*) w (circular), w white with variance sigma^2: the
    spectral density samples are |Omega| sigma^2 |DFT(h)|^2."""
    hp = np.zeros(shape)
    hp[tuple(slice(0, s) for s in h.shape)] = h
    H = np.fft.fftn(hp)
    return hp, np.prod(shape) * sigma ** 2 * np.abs(H) ** 2


def _noise(rng, hp, sigma, n):
    """n realisations of the circularly filtered white noise."""
    Hf = np.fft.fftn(hp)
    w = rng.normal(0.0, sigma, (n,) + hp.shape)
    axes = tuple(range(1, hp.ndim + 1))
    return np.real(np.fft.ifftn(np.fft.fftn(w, axes=axes) * Hf, axes=axes))


def test_autocovariance_closed_form():
    rng = np.random.default_rng(1)
    shape = (14, 11)
    h = rng.normal(size=(3, 4))
    sigma = 0.7
    hp, psd = _kernel_psd(shape, h, sigma)
    c = O.autocovariance(psd)
    # c(tau) = sigma^2 sum_t h(t) h(t + tau), indices modulo the shape
    ref = np.zeros(shape)
    for t0 in range(shape[0]):
        for t1 in range(shape[1]):
            s = 0.0
            for a in range(shape[0]):
                for b in range(shape[1]):
                    s += hp[a, b] * hp[(a + t0) % shape[0], (b + t1) % shape[1]]
            ref[t0, t1] = sigma ** 2 * s
    assert np.allclose(c, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # white spectrum: sigma^2 at zero displacement, zero elsewhere
    cw = O.autocovariance(np.full(shape, np.prod(shape) * sigma ** 2))
    expect = np.zeros(shape)
    expect[0, 0] = sigma ** 2
    assert np.allclose(cw, expect, atol=1e-15)


def _stage(shape, patch, search, psd, **kw):
    st = O.Stage(shape=shape, patch=patch, step=(1,) * len(shape), search=search,
                 noise="correlated", psd=psd, gamma=1.0, spatial="dct", **kw)
    return st


def test_corrected_ssd_is_unbiased_monte_carlo():
    """Every candidate's corrected score has expectation zero on pure noise
    (Prop. Gaussian SSD noise bias with gamma = 1); the uncorrected SSD does
    not, which shows the test can see the correction."""
    rng = np.random.default_rng(2)
    shape, patch, search = (10, 9), (3, 2), (4, 4)
    h = np.array([[1.0, 0.6, -0.2], [0.3, 0.5, 0.0]])   # anisotropic
    sigma = 1.0
    hp, psd = _kernel_psd(shape, h, sigma)
    # 4 x 4 window, interior references: 15 candidates, K = 16 holds them all
    st = _stage(shape, patch, search, psd, group_min=16, group_max=16, tau=1e30)
    refs = np.array([3 * shape[1] + 3, 4 * shape[1] + 4, 5 * shape[1] + 5], np.int64)
    R = 1500
    ys = _noise(rng, hp, sigma, R)
    sums, sums2 = {}, {}
    for y in ys:
        m, cnt, sc, _ = O.match(st, O.STAGE_HT, y, y, refs)
        assert (cnt == 16).all()
        for g in range(len(refs)):
            for k in range(1, 16):
                key = (g, int(m[g, k]))
                sums[key] = sums.get(key, 0.0) + sc[g, k]
                sums2[key] = sums2.get(key, 0.0) + sc[g, k] ** 2
    assert len(sums) == 3 * 15
    worst = 0.0
    for key, s in sums.items():
        mean = s / R
        sd = np.sqrt(max(sums2[key] / R - mean ** 2, 1e-30))
        worst = max(worst, abs(mean) / (sd / np.sqrt(R)))
    assert worst < 5.0, worst
    # the bias itself: the mean uncorrected SSD at a displacement is
    # 2 P (c(0) - c(Delta)), clearly non-zero here
    c = O.autocovariance(psd)
    P = 6
    ref = refs[0]
    r0, r1 = divmod(int(ref), shape[1])
    ssd = np.zeros(R)
    for i, y in enumerate(ys):
        p = y[r0:r0 + 3, r1:r1 + 2]
        q = y[r0 + 1:r0 + 4, r1 - 1:r1 + 1]
        ssd[i] = ((q - p) ** 2).sum()
    bias = 2 * P * (c[0, 0] - c[1, -1])
    assert abs(ssd.mean() - bias) < 5 * ssd.std() / np.sqrt(R)
    assert bias > 10 * ssd.std() / np.sqrt(R)


def _group_stage(shape, patch, psd, spatial, K):
    return O.Stage(shape=shape, patch=patch, step=(1,) * len(shape), search=(5,) * len(shape),
                   noise="correlated", psd=psd, spatial=spatial, group_min=K, group_max=K)


@pytest.mark.parametrize("spatial", ["dct", "bior1.5"])
def test_group_variance_monte_carlo(spatial):
    """Empirical variances of Y = T y_g over filtered-noise realisations
    match the propagated coefficient variances, for a group whose members
    overlap (shared voxels) and sit at different displacements."""
    rng = np.random.default_rng(3)
    shape, patch = (12, 10), (2, 4)
    h = np.array([[1.0, -0.5], [0.8, 0.25], [0.1, 0.4]])
    sigma = 0.5
    hp, psd = _kernel_psd(shape, h, sigma)
    K = 4
    org = np.array([2 * 10 + 3, 2 * 10 + 4, 3 * 10 + 3, 6 * 10 + 1], np.int32)
    st = _group_stage(shape, patch, psd, spatial, K)
    ys = _noise(rng, hp, sigma, 6000)
    _, var, _, _ = O.group_coeffs(st, O.STAGE_HT, ys[0], None, org)
    Ys = np.array([O.group_coeffs(st, O.STAGE_HT, y, None, org)[0] for y in ys])
    emp = Ys.var(axis=0)
    rel = np.sqrt(2.0 / len(ys))
    assert (var > 0).all()
    assert np.all(np.abs(emp / var - 1.0) < 5 * rel), np.abs(emp / var - 1.0).max()
    assert abs(np.mean(emp / var - 1.0)) < 5 * rel / np.sqrt(var.size)


def test_group_variance_explicit_kronecker():
    rng = np.random.default_rng(4)
    shape, patch = (9, 8), (3, 2)
    h = rng.normal(size=(2, 3))
    hp, psd = _kernel_psd(shape, h, 1.3)
    c = O.autocovariance(psd)
    K = 4
    org = np.array([0, 1, 9, 5 * 8 + 6], np.int32)   # overlapping and wrapped
    st = _group_stage(shape, patch, psd, "bior1.5", K)
    _, var, _, _ = O.group_coeffs(st, O.STAGE_HT, np.zeros(shape), None, org)
    T0, _ = O.spatial("bior1.5", patch[0])
    T1, _ = O.spatial("bior1.5", patch[1])
    T = np.kron(O.haar(K), np.kron(T0, T1))
    locs = []
    for o in org:
        a, b = divmod(int(o), shape[1])
        for i in range(patch[0]):
            for j in range(patch[1]):
                locs.append((a + i, b + j))
    n = len(locs)
    S = np.empty((n, n))
    for x in range(n):
        for z in range(n):
            S[x, z] = c[(locs[z][0] - locs[x][0]) % shape[0], (locs[z][1] - locs[x][1]) % shape[1]]
    ref = np.diag(T @ S @ T.T).reshape(K, -1)
    assert np.allclose(var, ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("stage", [O.STAGE_HT, O.STAGE_WIENER])
def test_white_spectrum_reduces_to_white_gaussian(stage):
    """A flat spectrum |Omega| sigma^2 gives c = sigma^2 delta: matching
    equals the white-Gaussian matching, and the filter equals white Gaussian
    noise with every plane exact (repeated voxels fully correlated)."""
    rng = np.random.default_rng(5)
    shape, patch, step, search = (26, 23), (4, 4), (3, 3), (9, 9)
    sigma = 0.2
    x = np.add.outer(np.sin(np.arange(26) / 3.0), np.cos(np.arange(23) / 4.0))
    y = x + rng.normal(0, sigma, shape)
    psd = np.full(shape, np.prod(shape) * sigma ** 2)
    white = O.plain_profile(shape, patch, step, search, noise="gaussian", sigma=sigma,
                            group=(8, 16))
    corr = O.plain_profile(shape, patch, step, search, noise="correlated", psd=psd,
                           group=(8, 16))
    w, cst = white[stage], corr[stage]
    w.k_exact = w.group_max
    refs = O.schedule(w, stage)
    src = y if stage == O.STAGE_HT else x
    mw, cw, sw, _ = O.match(w, stage, src, y, refs)
    mc, cc, sc, _ = O.match(cst, stage, src, y, refs)
    assert (mw == mc).all() and (cw == cc).all()
    assert np.allclose(sw, sc, rtol=1e-12, atol=1e-12)
    pil = None if stage == O.STAGE_HT else x
    pw, ww = O.filter(w, stage, y, pil, mw, cw)
    pc, wc = O.filter(cst, stage, y, pil, mc, cc)
    assert np.allclose(pw, pc, rtol=1e-10, atol=1e-12)
    assert np.allclose(ww, wc, rtol=1e-10)
    # and the diagonal white model differs once members overlap
    w.k_exact = 0
    pd, _ = O.filter(w, stage, y, pil, mw, cw)
    assert not np.allclose(pd, pc, rtol=1e-6, atol=1e-9)


def test_denoise_runs_on_correlated_noise():
    """End to end on filtered noise: finite output of the input's shape, and
    closer to the clean signal than the observation."""
    rng = np.random.default_rng(6)
    shape = (40, 36)
    x = np.add.outer(np.sin(np.arange(40) / 5.0), np.cos(np.arange(36) / 6.0))
    h = np.array([[1.0, 0.5], [0.5, 0.25]])
    hp, psd = _kernel_psd(shape, h, 0.15)
    y = x + _noise(rng, hp, 0.15, 1)[0]
    ht, wie = O.plain_profile(shape, (4, 4), (2, 2), (11, 11), noise="correlated", psd=psd,
                              group=(8, 16))
    pilot, out = O.denoise(ht, wie, y)
    assert out.shape == shape and np.isfinite(out).all()
    assert np.mean((out - x) ** 2) < 0.5 * np.mean((y - x) ** 2)
