"""Host-side checks of the HIP library (no GPU needed): the C ABI loads and
exports every declared symbol, host calls validate their arguments, and the
library's own schedule and tables agree with the oracle's independent ones."""
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2609_34622_amd as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "bmnd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:bmnd_status|const char\*)\s+(bmnd_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_version_and_presets():
    assert "gfx950" in B.bmnd_version()
    for nd in (1, 2, 3):
        p = B.bmnd_params_default(B.PRESET_PLAIN, nd)
        assert p.ht.group_max == 16 and p.wiener.group_max == 32
        assert p.ht.gamma == 3.0 and p.wiener.gamma == 0.0
        assert p.ht.spatial == B.SPATIAL["bior1.5"] and p.wiener.spatial == B.SPATIAL["dct"]
        s = B.bmnd_params_default(B.PRESET_STANDARD, nd)
        assert s.ht.k_exact == 4 and s.ht.weight_scope == B.SCOPE["patch"]
    with pytest.raises(B.BmndError):
        B.bmnd_params_default(7, 2)


@pytest.mark.parametrize("sched", ["generated", "balanced", "sparse", "off"])
@pytest.mark.parametrize("shape,patch,step", [((37, 41), (8, 8), (3, 3)),
                                              ((20, 18, 17), (4, 4, 4), (3, 3, 3)),
                                              ((1000,), (32,), (4,)),
                                              ((40, 1, 50), (8, 1, 8), (3, 1, 3)),
                                              ((9, 30), (5, 3), (2, 3))])
def test_library_schedule_equals_oracle(sched, shape, patch, step):
    sp = B.bmnd_params_default(0, len(shape)).ht
    B.set_axes(sp, patch=patch, step=step)
    sp.schedule = B.SCHED[sched]
    got = B.bmnd_reference_origins(B.geometry(shape), sp)
    st = O.Stage(shape=shape, patch=patch, step=step, search=(1,) * len(shape), schedule=sched)
    assert np.array_equal(got, O.schedule(st))


@pytest.mark.parametrize("kind", ["bior1.5", "dct", "identity"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 12, 16, 32])
def test_library_tables_equal_oracle(kind, n):
    T, U = B.bmnd_transform_matrices(kind, n)
    To, Uo = O.spatial(kind, n)
    assert np.abs(T - To).max() < 1e-13 and np.abs(U - Uo).max() < 1e-13
    # exact zeros must stay exact (hard thresholds of zero-variance
    # coefficients depend on them)
    assert np.array_equal(T == 0, To == 0) and np.array_equal(U == 0, Uo == 0)


def test_library_haar_and_kaiser_equal_oracle():
    for K in (1, 2, 4, 8, 16, 32):
        assert np.abs(B.bmnd_haar_matrix(K) - O.haar(K)).max() < 1e-14
    for n in (1, 4, 8, 32):
        assert np.abs(B.bmnd_kaiser_window(n, 2.0) - O.kaiser(n, 2.0)).max() < 1e-14


def _status(fn, *a):
    try:
        fn(*a)
    except B.BmndError as e:
        return e.status
    return B.OK


def test_validation_errors():
    g = B.geometry((64, 64))
    noise = B.poisson(0.1)
    p = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    assert B.bmnd_workspace_size(g, noise, p) > 0
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.ht.group_max = 12
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.wiener.gamma = 1.0
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.ht.weight_model = B.WEIGHT["risk"]
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    B.set_axes(bad.ht, patch=(65, 8))
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    B.set_axes(bad.ht, patch=(40, 40))
    assert _status(B.bmnd_workspace_size, B.geometry((64, 64)), noise, bad) in (B.E_UNSUPPORTED,)
    assert _status(B.bmnd_workspace_size, g, B.poisson(0.0), p) == B.E_ARG
    assert _status(B.bmnd_workspace_size, B.geometry((64,) * 5), noise,
                   B.bmnd_params_default(0, 5)) == B.E_UNSUPPORTED
    assert _status(B.bmnd_workspace_size, B.geometry((2 ** 16, 2 ** 16)), noise, p) == B.E_SHAPE
    g0 = B.geometry((64, 64))
    g0.batch = 0
    assert _status(B.bmnd_workspace_size, g0, noise, p) == B.E_SHAPE
    assert "batch" in B.lib().bmnd_last_error().decode()


def test_batch_workspace_layout():
    """Jobs go to four streams, longest first; a stream's jobs share its
    workspace, so the size is the sum of the per-stream maxima."""
    def job(shape, batch=1):
        j = B.Job()
        j.geom = B.geometry(shape, batch)
        j.noise = B.poisson(0.1)
        j.params = B.bmnd_params_default(B.PRESET_PLAIN, len(shape))
        return j

    one = [job((4096,)), job((64, 64)), job((24, 24, 24))]
    arr = (B.Job * 3)(*one)
    sizes = [B.bmnd_workspace_size(j.geom, j.noise, j.params) for j in one]
    assert B.bmnd_batch_workspace_size(arr) == sum(sizes)
    same = (B.Job * 6)(*[job((64, 64)) for _ in range(6)])
    assert B.bmnd_batch_workspace_size(same) == 4 * sizes[1]
    assert B.bmnd_batch_workspace_size((B.Job * 0)()) == 0
    bad = (B.Job * 2)(job((64, 64)), job((64, 64)))
    bad[1].noise = B.poisson(0.0)
    with pytest.raises(B.BmndError, match="job 1"):
        B.bmnd_batch_workspace_size(bad)


def test_poisson_metric_validation():
    g = B.geometry((64, 64))
    noise = B.poisson(0.1)
    p = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    assert p.ht.match_metric == B.METRIC_SSD and p.ht.match_policy == B.POLICY_FIXED
    assert (p.ht.match_t, p.ht.struct_beta, p.ht.struct_kappa) == (3.0, 0.1, 1.0)
    for m in (B.METRIC_DEVIANCE, B.METRIC_PEARSON, B.METRIC_ANSCOMBE):
        for pol in (B.POLICY_FIXED, B.POLICY_REFERENCE, B.POLICY_STANDARDIZED):
            ok = B.bmnd_params_default(B.PRESET_PLAIN, 2)
            ok.ht.match_metric, ok.ht.match_policy = m, pol
            assert B.bmnd_workspace_size(g, noise, ok) > 0
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.wiener.match_metric = B.METRIC_DEVIANCE           # HT-stage option only
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.ht.match_policy = B.POLICY_REFERENCE               # SSD uses the fixed policy
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.ht.match_metric = B.METRIC_PEARSON
    assert _status(B.bmnd_workspace_size, g, B.gaussian(0.1), bad) == B.E_ARG
    bad.ht.match_policy = B.POLICY_STANDARDIZED            # needs integral counts
    assert _status(B.bmnd_workspace_size, g, B.poisson(0.1, counts_integral=False), bad) == B.E_ARG
    bad.ht.match_t = -1.0
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad.ht.match_t, bad.ht.struct_kappa = 3.0, 0.0
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG
    bad.ht.struct_kappa, bad.ht.match_metric = 1.0, 7
    assert _status(B.bmnd_workspace_size, g, noise, bad) == B.E_ARG


@pytest.mark.parametrize("metric", ["deviance", "pearson", "anscombe"])
def test_library_moment_tables_equal_oracle(metric):
    code = {"deviance": B.METRIC_DEVIANCE, "pearson": B.METRIC_PEARSON,
            "anscombe": B.METRIC_ANSCOMBE}[metric]
    mu, v = B.bmnd_count_moments(code, 300)
    for n in list(range(0, 60)) + [127, 128, 299, 300]:
        mo, vo = O.count_moments(metric, n)
        assert abs(mu[n] - mo) <= 1e-12 * max(1.0, abs(mo)), n
        assert abs(v[n] - vo) <= 1e-11 * max(1.0, abs(vo)), n
    assert _status(B.bmnd_count_moments, B.METRIC_SSD, 10) == B.E_ARG
    assert _status(B.bmnd_count_moments, code, B.MOMENT_MAX_COUNT + 1) == B.E_ARG


def test_correlated_noise_validation():
    """Table sizes of the correlated model and the host-side checks of a
    noise model's table pointer (no device work)."""
    g = B.geometry((64, 48))
    p = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    n1 = B.bmnd_correlated_size(g, p)
    assert n1 > 0 and n1 % 256 == 0
    # batch does not change the tables; a wider window needs more
    assert B.bmnd_correlated_size(B.geometry((64, 48), batch=3), p) == n1
    wide = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    for sp in (wide.ht, wide.wiener):
        B.set_axes(sp, search=(31, 31))
    assert B.bmnd_correlated_size(g, wide) > n1
    # a pointer that no prepare call wrote is refused before any launch
    fake = B.Noise()
    fake.kind = B.NOISE_CORRELATED
    fake.d_corr = 4096
    assert _status(B.bmnd_workspace_size, g, fake, p) == B.E_ARG
    fake.d_corr = None
    assert _status(B.bmnd_workspace_size, g, fake, p) == B.E_ARG
    bad = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    bad.ht.group_max = 3
    assert _status(B.bmnd_correlated_size, g, bad) == B.E_ARG


def test_serving_work_cap_rule():
    """The serving admission rule: the work estimate grows with the array
    and the window, and a busy device admits only within the cap."""
    from paper_2609_34622_amd import serving

    def req(shape, ndim):
        return serving.Request(0, 0.0, np.zeros(shape, np.float32), 0.1,
                               serving.default_params(ndim, False))

    small, big = req((64, 64), 2), req((512, 512), 2)
    assert serving.request_work(big) > 50 * serving.request_work(small)
    one_d = req((65536,), 1)
    assert serving.request_work(one_d) > 0
    w = serving.request_work(big)
    assert serving.admits(0.0, w, w / 10, busy=False)      # idle: always
    assert not serving.admits(w, w, w, busy=True)         # two large ones: no
    assert serving.admits(w / 4, w / 4, w, busy=True)     # small beside small: yes
    assert serving.admits(w, w, None, busy=True)          # no cap


def test_request_bytes_and_budget():
    """bmnd_request_bytes: arrays plus workspace; E_BUDGET beyond a budget."""
    shape = (64, 48)
    p = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    geom, noise = B.geometry(shape, 3), B.poisson(0.1)
    need = B.bmnd_request_bytes(geom, noise, p)
    assert need == B.bmnd_workspace_size(geom, noise, p) + 2 * 4 * 3 * 64 * 48
    assert B.bmnd_request_bytes(geom, noise, p, need) == need
    with pytest.raises(B.BmndError) as e:
        B.bmnd_request_bytes(geom, noise, p, need - 1)
    assert e.value.status == B.E_BUDGET


def test_up_to_eight_axes_with_at_most_four_wide():
    """ndim up to 8: singleton axes are dropped for the kernels (the sizes
    equal those of the squeezed array's), more than 4 wide axes are refused,
    and the schedule is still built on all axes."""
    p5 = B.bmnd_params_default(B.PRESET_PLAIN, 5)
    for sp in (p5.ht, p5.wiener):
        B.set_axes(sp, patch=(1, 4, 1, 4, 4), step=(1, 3, 1, 3, 3), search=(1, 7, 1, 7, 7))
    p3 = B.bmnd_params_default(B.PRESET_PLAIN, 3)
    for sp in (p3.ht, p3.wiener):
        B.set_axes(sp, patch=(4, 4, 4), step=(3, 3, 3), search=(7, 7, 7))
    n = B.poisson(0.1)
    g5, g3 = B.geometry((1, 20, 1, 18, 16)), B.geometry((20, 18, 16))
    assert B.bmnd_workspace_size(g5, n, p5) > 0
    assert B.bmnd_match_workspace_size(g5, p5.ht) == B.bmnd_match_workspace_size(g3, p3.ht)
    # the generated schedule sees the singleton axis between axes 1 and 3
    o5 = B.bmnd_reference_origins(g5, p5.ht)
    st = O.Stage(shape=(1, 20, 1, 18, 16), patch=(1, 4, 1, 4, 4), step=(1, 3, 1, 3, 3),
                 search=(1, 7, 1, 7, 7))
    assert np.array_equal(o5, O.schedule(st))
    p8 = B.bmnd_params_default(B.PRESET_PLAIN, 8)
    for sp in (p8.ht, p8.wiener):
        B.set_axes(sp, patch=(2,) * 5 + (1,) * 3, step=(1,) * 8, search=(3,) * 5 + (1,) * 3)
    with pytest.raises(B.BmndError) as e:
        B.bmnd_workspace_size(B.geometry((4, 4, 4, 4, 4, 1, 1, 1)), n, p8)
    assert e.value.status == B.E_UNSUPPORTED
    for sp in (p8.ht, p8.wiener):
        B.set_axes(sp, patch=(1,) + (2,) * 4 + (1,) * 3, step=(1,) * 8,
                   search=(1,) + (3,) * 4 + (1,) * 3)
    assert B.bmnd_workspace_size(B.geometry((1, 4, 4, 4, 4, 1, 1, 1)), n, p8) > 0
