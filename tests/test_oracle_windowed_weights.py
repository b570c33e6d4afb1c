"""Pins of the oracle's windowed synthesized-domain aggregation weights
(Def. windowed synthesis metrics, Prop. windowed transmitted-noise energy,
Def. windowed synthesized-domain weighting models)."""
import numpy as np
import pytest

import oracle as O


def _group(st, stage=O.STAGE_HT, seed=3):
    rng = np.random.default_rng(seed)
    y = (rng.poisson(4.0, size=st.shape) * st.s_p).astype(np.float64)
    K = 4
    org = np.array([0, 3, 17, 40], np.int32)
    pilot = y * 0.9 if stage == O.STAGE_WIENER else None
    return y, pilot, org, K


@pytest.mark.parametrize("model,scope", [("classic", "group"), ("variance", "group"),
                                         ("classic", "patch"), ("variance", "patch")])
def test_unitary_synthesis_and_flat_window_reduce_to_coefficient_domain(model, scope):
    # the paper: with unitary inverse synthesis and a constant window H = I,
    # so the windowed models reduce to the coefficient-domain ones
    base = dict(shape=(12, 10), patch=(4, 4), step=(2, 2), search=(5, 5), s_p=0.25,
                spatial="dct", kaiser_beta=0.0, weight_model=model, weight_scope=scope)
    st_c = O.Stage(**base)
    st_w = O.Stage(**base, weight_domain="windowed")
    y, pil, org, K = _group(st_c)
    _, _, _, wc = O.group_coeffs(st_c, O.STAGE_HT, y, pil, org)
    _, _, _, ww = O.group_coeffs(st_w, O.STAGE_HT, y, pil, org)
    assert np.allclose(wc, ww, rtol=1e-12)


@pytest.mark.parametrize("stage,model,spatial", [(O.STAGE_HT, "variance", "bior1.5"),
                                                 (O.STAGE_WIENER, "variance", "dct"),
                                                 (O.STAGE_HT, "classic", "bior1.5")])
def test_windowed_surrogate_is_the_transmitted_noise_energy(stage, model, spatial):
    # Prop. windowed transmitted-noise energy: E||L F N||^2 = tr(H F Sigma F^H)
    # for N ~ N(0, Sigma); Monte Carlo with L = W_g U_g built densely here
    # from the Haar, spatial synthesis and Kaiser matrices
    shrink = "wiener" if stage == O.STAGE_WIENER else "hard"
    st = O.Stage(shape=(12, 10), patch=(4, 4), step=(2, 2), search=(5, 5), s_p=0.25,
                 spatial=spatial, shrink=shrink, weight_model=model, weight_scope="group",
                 weight_domain="windowed", kaiser_beta=2.0, lam=1.5)
    y, pil, org, K = _group(st, stage)
    Y, var, Cc, w = O.group_coeffs(st, stage, y, pil, org)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(Y != 0, Cc / Y, 0.0).ravel()
    sig2 = np.maximum(var.ravel(), 0.0) if model == "variance" else np.ones(f.size)
    _, U0 = O.spatial(spatial, 4)
    Ug = np.kron(O.haar(K).T, np.kron(U0, U0))
    win = np.outer(O.kaiser(4, 2.0), O.kaiser(4, 2.0)).ravel()
    L = np.tile(win, K)[:, None] * Ug
    rng = np.random.default_rng(11)
    n = rng.normal(size=(f.size, 40000)) * np.sqrt(sig2)[:, None]
    e = ((L @ (f[:, None] * n)) ** 2).sum(axis=0)
    mc, se = e.mean(), e.std() / np.sqrt(e.size)
    R = 1.0 / w[0]
    assert abs(R - mc) <= 5 * se + 1e-12, (R, mc, se)
    # and exactly the trace of the dense metric
    H = L.T @ L
    assert abs(R - float(np.sum(np.diag(H) * f * f * sig2))) <= 1e-10 * R


def test_patch_scope_splits_the_group_metric():
    # H_g = sum_j H_{g,j}: the patch surrogates sum to the group surrogate
    base = dict(shape=(12, 10), patch=(4, 4), step=(2, 2), search=(5, 5), s_p=0.25,
                spatial="bior1.5", kaiser_beta=2.0, weight_model="variance",
                weight_domain="windowed")
    st_g = O.Stage(**base, weight_scope="group")
    st_p = O.Stage(**base, weight_scope="patch")
    y, pil, org, K = _group(st_g)
    _, _, _, wg = O.group_coeffs(st_g, O.STAGE_HT, y, pil, org)
    _, _, _, wp = O.group_coeffs(st_p, O.STAGE_HT, y, pil, org)
    assert abs(np.sum(1.0 / wp) - 1.0 / wg[0]) <= 1e-10 / wg[0]
