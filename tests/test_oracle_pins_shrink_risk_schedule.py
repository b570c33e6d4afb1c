"""Pins of four oracle functions against what the paper and the mathematics
fix, each built independently of the oracle's code here:

- the soft threshold (eq. soft-threshold) and its attenuation weights, on a
  K = 2 group whose transform is assembled densely in this file (Haar by
  hand, DCT from scipy), checked as the proximal operator of lambda sigma |.|
  by direct minimisation;
- the Wiener risk weights (eq. diagonal-wiener-risk and the risk weighting
  model, coefficient and windowed synthesized domains, group and patch
  scope), against the closed form on the dense transform and against a
  Monte-Carlo estimate of the risk of the diagonal Wiener filter under the
  diagonal signal model;
- the balanced reference schedule (Def. balanced reference schedule), against
  hand-worked origin sets and an independent vectorised enumeration;
- the hard threshold at zero variance (eq. hard-threshold with sigma_k = 0):
  coefficients that are 0 in exact arithmetic are dropped whatever their
  rounding residue, nonzero ones are kept.
"""
import os

import numpy as np
import pytest
import scipy.fft
import scipy.optimize

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")

H2 = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)   # orthonormal Haar, K = 2


def _dct_matrix(n):
    # orthonormal DCT-II as scipy computes it, column by column
    return scipy.fft.dct(np.eye(n), norm="ortho", axis=0)


def _dense_T(n):
    Tsp = np.kron(_dct_matrix(n), _dct_matrix(n))   # 2-D patch, C-order samples
    return np.kron(H2, Tsp), Tsp


def _group(shape, org, n, arr):
    """Group vector (member-major, C-order samples) of the n x n patches at
    the given origins (lin)."""
    rows = []
    for o in org:
        r, c = divmod(int(o), shape[1])
        rows.append(arr[r:r + n, c:c + n].ravel())
    return np.concatenate(rows)


SHAPE = (9, 10)
N = 4
ORG = np.array([11, 25], np.int32)   # (1, 1) and (2, 5)


def _poisson_array(seed, s_p, lam=5.0):
    rng = np.random.default_rng(seed)
    return rng.poisson(lam, size=SHAPE).astype(np.float64) * s_p


# ------------------------------------------------------------ soft threshold

@pytest.mark.parametrize("lam", [0.7, 1.5])
def test_soft_threshold_is_the_prox_of_lambda_sigma_abs(lam):
    s_p = 0.5
    y = _poisson_array(1, s_p)
    st = O.Stage(shape=SHAPE, patch=(N, N), step=(3, 3), search=(5, 5), s_p=s_p,
                 spatial="dct", shrink="soft", lam=lam, kaiser_beta=0.0)
    Y, var, Cc, w = O.group_coeffs(st, O.STAGE_HT, y, None, ORG)
    T, _ = _dense_T(N)
    yg = _group(SHAPE, ORG, N, y)
    Yd = T @ yg
    sig2 = (T * T) @ (s_p * np.maximum(yg, 0.0))   # diagonal Poisson variance propagation
    assert np.allclose(Y.ravel(), Yd, rtol=0, atol=1e-12 * np.abs(Yd).max())
    assert np.allclose(var.ravel(), sig2, rtol=1e-12, atol=1e-15)
    # each shrunk coefficient minimises 1/2 (c - Y)^2 + lambda sigma |c|
    sig = np.sqrt(sig2)
    for k in range(Yd.size):
        f = lambda c: 0.5 * (c - Yd[k]) ** 2 + lam * sig[k] * abs(c)
        lo, hi = -abs(Yd[k]) - 1.0, abs(Yd[k]) + 1.0
        best = scipy.optimize.minimize_scalar(f, bounds=(lo, hi), method="bounded",
                                              options={"xatol": 1e-10}).x
        assert abs(Cc.ravel()[k] - best) <= 1e-7 * (abs(Yd[k]) + 1.0), k
    # the test distinguishes lambda sigma from lambda sigma^2: some coefficients
    # survive with sigma != 1 on both sides of 1
    kept = np.abs(Cc.ravel()) > 0
    assert kept.any() and (~kept).any()
    assert (sig[kept] > 1.0).any() or (sig[kept] < 1.0).any()


@pytest.mark.parametrize("model,scope", [("classic", "group"), ("variance", "group"),
                                         ("variance", "patch")])
def test_soft_threshold_attenuation_weights_by_hand(model, scope):
    # weights from the attenuation a_k = |C_k| / |Y_k| (the coefficient-domain
    # hard-thresholding weighting model with the soft threshold's gain)
    s_p, lam = 0.5, 1.5
    y = _poisson_array(2, s_p)
    st = O.Stage(shape=SHAPE, patch=(N, N), step=(3, 3), search=(5, 5), s_p=s_p,
                 spatial="dct", shrink="soft", lam=lam, kaiser_beta=0.0,
                 weight_model=model, weight_scope=scope)
    _, _, _, w = O.group_coeffs(st, O.STAGE_HT, y, None, ORG)
    T, _ = _dense_T(N)
    yg = _group(SHAPE, ORG, N, y)
    Yd = T @ yg
    sig2 = (T * T) @ (s_p * np.maximum(yg, 0.0))
    m = np.maximum(np.abs(Yd) - lam * np.sqrt(sig2), 0.0)
    a = np.where(Yd != 0, m / np.abs(Yd), 0.0)
    t = a * a if model == "classic" else a * a * sig2
    r = t.reshape(2, -1).sum(axis=1)     # per Haar plane
    if scope == "group":
        want = np.full(2, 1.0 / r.sum())
    else:
        want = 1.0 / ((H2 ** 2).T @ r)   # R_j = sum_l H_lj^2 r_l
    assert np.allclose(w, want, rtol=1e-12)


# -------------------------------------------------------------- risk weights

def _wiener_setup(seed=3, power_a=1.0, s_v=0.4):
    s_p = 0.25
    rng = np.random.default_rng(seed)
    y = rng.poisson(6.0, size=SHAPE).astype(np.float64) * s_p
    pilot = np.clip(y + rng.normal(0.0, 0.3, size=SHAPE), 0.0, None)
    T, Tsp = _dense_T(N)
    pg = _group(SHAPE, ORG, N, pilot)
    G = T @ pg                                          # pilot coefficients Gamma
    sig2 = (T * T) @ (s_p * np.maximum(pg, 0.0))        # variance map from the pilot
    S = np.maximum(G * G - power_a * sig2, 0.0)         # eq. pilot-power-family
    den = S + s_v * sig2
    g = np.where(den > 0, S / np.where(den > 0, den, 1.0), 0.0)   # eq. wiener-gain
    return s_p, y, pilot, sig2, S, g, Tsp


@pytest.mark.parametrize("scope", ["group", "patch"])
def test_risk_weights_closed_form(scope):
    s_p, y, pilot, sig2, S, g, _ = _wiener_setup()
    st = O.Stage(shape=SHAPE, patch=(N, N), step=(3, 3), search=(5, 5), s_p=s_p,
                 spatial="dct", shrink="wiener", power_a=1.0, s_v=0.4, kaiser_beta=0.0,
                 weight_model="risk", weight_scope=scope)
    _, _, _, w = O.group_coeffs(st, O.STAGE_WIENER, y, pilot, ORG)
    risk = g * g * sig2 + (1.0 - g) ** 2 * S             # eq. diagonal-wiener-risk
    r = risk.reshape(2, -1).sum(axis=1)
    want = np.full(2, 1.0 / r.sum()) if scope == "group" else 1.0 / ((H2 ** 2).T @ r)
    assert np.allclose(w, want, rtol=1e-12)
    # power_a = 1 makes S differ from Gamma^2, so the pin tells them apart
    assert not np.allclose(S, S + sig2)


def test_risk_is_the_mse_of_the_diagonal_wiener_filter():
    # with a signal theta of second moment S (random signs: E theta theta^T =
    # diag(S), Remark diagonal signal model) and noise of variance sigma^2,
    # E ||G (theta + n) - theta||^2 = sum G^2 sigma^2 + (1 - G)^2 S
    s_p, y, pilot, sig2, S, g, _ = _wiener_setup(seed=4)
    st = O.Stage(shape=SHAPE, patch=(N, N), step=(3, 3), search=(5, 5), s_p=s_p,
                 spatial="dct", shrink="wiener", power_a=1.0, s_v=0.4, kaiser_beta=0.0,
                 weight_model="risk", weight_scope="group")
    _, _, _, w = O.group_coeffs(st, O.STAGE_WIENER, y, pilot, ORG)
    rng = np.random.default_rng(12)
    M = 200000
    theta = np.sqrt(S)[:, None] * rng.choice([-1.0, 1.0], size=(S.size, M))
    n = np.sqrt(sig2)[:, None] * rng.normal(size=(S.size, M))
    e = ((g[:, None] * (theta + n) - theta) ** 2).sum(axis=0)
    mc, se = e.mean(), e.std() / np.sqrt(M)
    R = 1.0 / w[0]
    assert abs(R - mc) <= 5 * se, (R, mc, se)


@pytest.mark.parametrize("scope", ["group", "patch"])
def test_windowed_risk_is_the_windowed_synthesis_mse(scope):
    # windowed synthesized domain (Def. windowed synthesized-domain weighting
    # models, with the diagonal signal and noise models): the surrogate of
    # member j is E ||W (U_g (G (theta + n) - theta))_j||^2; Monte Carlo
    # through the dense synthesis L = W U_g
    s_p, y, pilot, sig2, S, g, Tsp = _wiener_setup(seed=5)
    st = O.Stage(shape=SHAPE, patch=(N, N), step=(3, 3), search=(5, 5), s_p=s_p,
                 spatial="dct", shrink="wiener", power_a=1.0, s_v=0.4, kaiser_beta=2.0,
                 weight_model="risk", weight_scope=scope, weight_domain="windowed")
    _, _, _, w = O.group_coeffs(st, O.STAGE_WIENER, y, pilot, ORG)
    Ug = np.kron(H2.T, np.linalg.inv(Tsp))
    win = np.outer(np.kaiser(N, 2.0), np.kaiser(N, 2.0)).ravel()
    L = np.tile(win, 2)[:, None] * Ug
    rng = np.random.default_rng(13)
    M = 100000
    theta = np.sqrt(S)[:, None] * rng.choice([-1.0, 1.0], size=(S.size, M))
    n = np.sqrt(sig2)[:, None] * rng.normal(size=(S.size, M))
    err = L @ (g[:, None] * (theta + n) - theta)          # synthesized, windowed error
    P = N * N
    per_member = (err.reshape(2, P, M) ** 2).sum(axis=1)    # [member, sample]
    if scope == "group":
        e = per_member.sum(axis=0)
        mc, se = e.mean(), e.std() / np.sqrt(M)
        assert abs(1.0 / w[0] - mc) <= 5 * se, (1.0 / w[0], mc, se)
    else:
        for j in range(2):
            e = per_member[j]
            mc, se = e.mean(), e.std() / np.sqrt(M)
            assert abs(1.0 / w[j] - mc) <= 5 * se, (j, 1.0 / w[j], mc, se)


# ---------------------------------------------------------- balanced schedule

def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_balanced_schedule_hand_worked():
    for row in _rows("balanced_hand.txt"):
        shape = tuple(int(v) for v in row[0].split(","))
        patch = tuple(int(v) for v in row[1].split(","))
        step = tuple(int(v) for v in row[2].split(","))
        st = O.Stage(shape=shape, patch=patch, step=step, search=(1,) * len(shape),
                     schedule="balanced", shift_density=2.0, passes=2)
        assert O.schedule(st).tolist() == [int(v) for v in row[3:]], row


def _shift_list(j, h, rho):
    # eq. number-shifts and eq. candidate-shift-list
    n = min(j, max(1, int(np.ceil(rho * (j - 1) / h - 1e-12))))
    if n == 1:
        return np.zeros(1, np.int64)
    return np.floor(np.arange(n) * (j - 1) / (n - 1) + 0.5).astype(np.int64)


def balanced_origins(shape, patch, step, rho, passes):
    """Independent vectorised enumeration of Def. balanced reference schedule
    over all slot tuples at once."""
    D = len(shape)
    ell = np.array(shape) - np.array(patch)
    Z = -(-ell // np.array(step)) + 1
    grids = np.meshgrid(*[np.arange(z) for z in Z], indexing="ij")
    q = np.stack([g.ravel() for g in grids])                 # [D, slots]
    Q = q.sum(axis=0)
    strides = np.cumprod((list(shape[1:]) + [1])[::-1])[::-1]
    out = []
    for k in range(passes):
        lin = np.zeros(q.shape[1], np.int64)
        for d in range(D):
            S = _shift_list(patch[d], step[d], rho)
            o = S[(k + Q - q[d]) % len(S)]
            slot = np.minimum(q[d] * step[d], ell[d])
            r = np.clip(slot - o, 0, ell[d])
            r = np.where(q[d] == Z[d] - 1, ell[d], r)
            lin += r * strides[d]
        out.append(lin)
    return np.unique(np.concatenate(out))


@pytest.mark.parametrize("shape,patch,step,rho,passes", [
    ((128, 128), (8, 8), (3, 3), 2.0, 2),
    ((1024, 1024), (8, 8), (3, 3), 2.0, 2),
    ((256, 256, 128), (4, 4, 4), (3, 3, 3), 2.0, 2),
    ((65536,), (32,), (4,), 2.0, 2),
    ((37, 41), (8, 8), (3, 3), 4.0, 3),
    ((20, 18, 17), (4, 5, 4), (3, 2, 3), 2.0, 2),
    ((9, 7, 8, 6), (3, 3, 4, 2), (2, 2, 3, 1), 2.0, 3),
])
def test_balanced_schedule_equals_independent_enumeration(shape, patch, step, rho, passes):
    st = O.Stage(shape=shape, patch=patch, step=step, search=(1,) * len(shape),
                 schedule="balanced", shift_density=rho, passes=passes)
    got = O.schedule(st)
    want = balanced_origins(shape, patch, step, rho, passes)
    assert np.array_equal(got, want)


# ------------------------------------------------ zero-variance hard threshold

@pytest.mark.parametrize("spatial", ["bior1.5", "dct"])
@pytest.mark.parametrize("K", [2, 4, 8])
def test_zero_variance_exact_zeros_are_dropped(spatial, K):
    # a constant negative group: the Poisson variance map [y]_+ is 0, so every
    # threshold is 0; in exact arithmetic only the DC coefficient of the
    # scaling row is nonzero (detail rows of H and the high-pass rows of the
    # spatial transform sum to zero), so exactly one coefficient is kept and
    # the classic weight is 1 / 1 -- rounding residues of the others must not
    # count as kept coefficients
    shape = (12, 40)
    y = np.full(shape, -0.37)
    org = np.arange(K, dtype=np.int32) * 4
    st = O.Stage(shape=shape, patch=(8, 8), step=(3, 3), search=(5, 5), s_p=0.5,
                 spatial=spatial, shrink="hard", lam=3.0, kaiser_beta=2.0)
    Y, var, Cc, w = O.group_coeffs(st, O.STAGE_HT, y, None, org)
    assert np.all(var == 0.0)
    assert np.count_nonzero(Cc) == 1
    assert np.allclose(w, 1.0, rtol=0, atol=0)


def test_zero_variance_nonzero_coefficients_are_kept():
    # a negative ramp: zero variance everywhere, and every coefficient whose
    # magnitude is well above the rounding scale of its terms is kept
    shape = (12, 40)
    yy, xx = np.meshgrid(np.arange(12), np.arange(40), indexing="ij")
    y = -1.0 - 0.01 * xx - 0.02 * yy
    org = np.array([0, 5], np.int32)
    st = O.Stage(shape=shape, patch=(8, 8), step=(3, 3), search=(5, 5), s_p=0.5,
                 spatial="dct", shrink="hard", lam=3.0)
    Y, var, Cc, w = O.group_coeffs(st, O.STAGE_HT, y, None, org)
    assert np.all(var == 0.0)
    big = np.abs(Y) > 1e-6 * np.abs(Y).max()
    assert np.array_equal(Cc != 0, big)
    assert np.isclose(w[0], 1.0 / big.sum(), rtol=1e-12)
