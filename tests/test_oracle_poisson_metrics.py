"""Pins of the oracle's Poisson-likelihood matching metrics and their
finite-count calibration (section Metrics; subsection Exact Finite-Count
Moment Calibration), each against something other than the oracle's own
formula: closed forms the paper proves, the Poisson likelihood from scipy,
the paper's worked numbers, exact enumeration of the conditional null."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O

METRICS = ["deviance", "pearson", "anscombe"]


def test_zero_pooled_count_has_zero_moments():
    # Prop. universal finite-count moments: at n = 0 the only allocation
    # is (0, 0), whose contribution is zero
    for m in METRICS:
        assert O.count_moments(m, 0) == (0.0, 0.0)
        assert O.phi(m, 0, 0) == 0.0


@pytest.mark.parametrize("n", list(range(1, 41)) + [97, 250])
def test_pearson_moments_closed_form(n):
    # Prop. exact Pearson moments: mu = 1, v = 2 - 2/n for n >= 1
    mu, v = O.count_moments("pearson", n)
    assert abs(mu - 1.0) < 1e-12
    assert abs(v - (2.0 - 2.0 / n)) < 1e-11


@pytest.mark.parametrize("r,c", [(0, 1), (1, 0), (3, 1), (5, 5), (7, 2), (0, 12), (20, 31)])
def test_deviance_is_the_poisson_likelihood_ratio(r, c):
    # Prop. deviance as likelihood ratio: -2 log of the equal-rate maximum
    # likelihood over the separate-rate one
    lam0 = (r + c) / 2.0
    l0 = stats.poisson.logpmf(r, lam0) + stats.poisson.logpmf(c, lam0)
    l1 = stats.poisson.logpmf(r, r) + stats.poisson.logpmf(c, c)
    assert abs(O.phi("deviance", r, c) - (-2.0 * (l0 - l1))) < 1e-10


@pytest.mark.parametrize("m,delta", [(1e4, 10.0), (1e4, 40.0), (1e6, 100.0)])
def test_common_high_count_limit(m, delta):
    # Thm. common high-count limit: phi = delta^2 / (2m) + o(delta^2 / m);
    # Pearson exactly; the deviance's next term is delta^4 / (48 m^3)
    r, c = m + delta / 2, m - delta / 2
    lead = delta ** 2 / (2 * m)
    assert abs(O.phi("pearson", r, c) - lead) <= 1e-12 * lead
    dev = O.phi("deviance", r, c)
    # (plus the FP64 cancellation of the two O(m t) terms of the formula)
    assert abs(dev - lead - delta ** 4 / (48 * m ** 3)) <= 10 * delta ** 6 / m ** 5 + 1e-15 * (r + c)
    assert abs(O.phi("anscombe", r, c) - lead) <= 2 * (delta / m) * lead


def test_anscombe_small_count_breakdown():
    # Example (breakdown of the Anscombe approximation): for K ~ Poi(1),
    # E[A(K)] ~ 2.18691 and Var A(K) ~ 0.717443, with A(k) = A(0) +
    # sqrt(2 phi_A(k, 0)) (A is increasing)
    a0 = 2.0 * math.sqrt(3.0 / 8.0)
    ks = np.arange(0, 60)
    A = np.array([a0 + math.sqrt(2.0 * O.phi("anscombe", k, 0)) for k in ks])
    w = stats.poisson.pmf(ks, 1.0)
    ea = float((w * A).sum())
    assert abs(float((w * A * A).sum()) - 5.5) < 1e-12
    assert abs(ea - 2.18691) < 5e-6
    assert abs(5.5 - ea * ea - 0.717443) < 5e-6


@pytest.mark.parametrize("metric", METRICS)
@pytest.mark.parametrize("n", [1, 2, 5, 13, 40])
def test_moments_against_binomial_enumeration(metric, n):
    # Lemma conditional Poisson splitting: r | r + c = n ~ Bin(n, 1/2); the
    # oracle's moments against scipy's binomial weights over the oracle's
    # per-entry contributions
    x = np.arange(n + 1)
    w = stats.binom.pmf(x, n, 0.5)
    f = np.array([O.phi(metric, k, n - k) for k in x])
    mu, v = O.count_moments(metric, n)
    assert abs(mu - (w * f).sum()) < 1e-11
    assert abs(v - ((w * f * f).sum() - (w * f).sum() ** 2)) < 1e-10


@pytest.mark.parametrize("metric", METRICS)
def test_standardized_distance_null_moments(metric):
    # Cor. standardized null moments: given the pooled counts, Z has mean 0
    # and variance 1 when the entries are conditionally independent; exact
    # enumeration of every allocation
    n = [2, 5, 0, 3]
    e1 = e2 = 0.0
    for xs in itertools.product(*[range(k + 1) for k in n]):
        w = np.prod([stats.binom.pmf(x, k, 0.5) for x, k in zip(xs, n)])
        r = np.array(xs, float)
        c = np.array(n, float) - r
        z, th = O.pair_score(metric, "standardized", r, c, t=2.5)
        assert th == 2.5
        e1 += w * z
        e2 += w * z * z
    assert abs(e1) < 1e-12
    assert abs(e2 - 1.0) < 1e-12


def test_reference_threshold_pearson_closed_form():
    # Def. reference finite-count threshold with Pearson's closed-form
    # moments at n = 2 r_i
    r = np.array([0.0, 1.0, 3.0, 2.0, 0.0, 6.0])
    c = np.array([1.0, 0.0, 2.0, 2.0, 0.0, 4.0])
    P, t, beta, kappa = len(r), 2.0, 0.1, 1.5
    n = 2 * r
    mu = np.where(n > 0, 1.0, 0.0)
    v = np.where(n > 0, 2.0 - 2.0 / np.maximum(n, 1), 0.0)
    expect = mu.mean() + t * math.sqrt(v.sum() / P ** 2) + beta * r.mean() ** kappa
    d, th = O.pair_score("pearson", "reference", r, c, t=t, beta=beta, kappa=kappa)
    assert abs(th - expect) < 1e-12
    s = sum((ci - ri) ** 2 / (ri + ci) for ri, ci in zip(r, c) if ri + ci > 0)
    assert abs(d - s / P) < 1e-12


def test_fixed_threshold_is_the_high_count_calibration():
    # reading: the fixed policy uses the high-count mean 1 and variance 2 per
    # entry, so the patch threshold is 1 + t sqrt(2 / P)
    for P in (4, 32, 64):
        _, th = O.pair_score("deviance", "fixed", np.ones(P), np.ones(P), t=3.0)
        assert abs(th - (1.0 + 3.0 * math.sqrt(2.0 / P))) < 1e-14


@pytest.mark.parametrize("metric,policy", [(m, p) for m in METRICS
                                           for p in ("fixed", "reference", "standardized")])
def test_match_lists_follow_pair_scores(metric, policy):
    # the grouping step on a tiny 2-D Poisson image: reference first, then
    # the accepted candidates by (score, lin), group size from the accepted
    # count, every score from the pinned pair function
    rng = np.random.default_rng(7)
    shape, patch, search = (9, 8), (3, 2), (5, 5)
    s_p = 0.25
    y = (rng.poisson(3.0, size=shape) * s_p).astype(np.float64)
    st = O.Stage(shape=shape, patch=patch, step=(2, 2), search=search, group_max=8, gamma=3.0,
                 s_p=s_p, metric=metric, policy=policy, match_t=0.5)
    refs = O.schedule(st)
    m, cnt, sc, acc = O.match(st, O.STAGE_HT, y, y, refs)
    kap = np.rint(y / s_p)
    for g, r in enumerate(refs):
        r0, r1 = divmod(int(r), shape[1])
        cands = []
        for c0 in range(max(r0 - 2, 0), min(r0 + 2, shape[0] - patch[0]) + 1):
            for c1 in range(max(r1 - 2, 0), min(r1 + 2, shape[1] - patch[1]) + 1):
                lin = c0 * shape[1] + c1
                if lin == r:
                    continue
                pr = kap[r0:r0 + patch[0], r1:r1 + patch[1]].ravel()
                pc = kap[c0:c0 + patch[0], c1:c1 + patch[1]].ravel()
                d, th = O.pair_score(metric, policy, pr, pc, t=0.5)
                cands.append((d, lin, th))
        cands.sort()
        nacc = sum(1 for d, _, th in cands if d < th)
        assert acc[g] == nacc
        K = 1 << (min(1 + nacc, 8).bit_length() - 1)
        K = max(K, 2)
        K = min(K, 1 << ((1 + len(cands)).bit_length() - 1))
        assert cnt[g] == K
        assert m[g, 0] == r
        assert list(m[g, 1:K]) == [lin for _, lin, _ in cands[:K - 1]]
