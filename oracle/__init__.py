"""FP64 CPU oracle of the BMND hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The GPU library never imports it, and
this module never imports the GPU package: the two share no code.

The arithmetic lives in ``bmnd_oracle.c`` (plain C99, double precision,
single-threaded); this file only builds it with gcc and marshals numpy arrays
through ctypes.  Each C function cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmnd_oracle.c")
_LIB = os.path.join(_HERE, "libbmnd_oracle.so")

MAXD = 8
SCHED = {"generated": 0, "balanced": 1, "sparse": 2, "off": 3}
SPATIAL = {"identity": 0, "dct": 1, "bior1.5": 2}
SHRINK = {"hard": 0, "soft": 1, "wiener": 2}
WMODEL = {"classic": 0, "variance": 1, "risk": 2}
WSCOPE = {"group": 0, "patch": 1}
NOISE = {"gaussian": 0, "poisson": 1, "correlated": 2}
METRIC = {"ssd": 0, "deviance": 1, "pearson": 2, "anscombe": 3}
POLICY = {"fixed": 0, "reference": 1, "standardized": 2}
WDOMAIN = {"coefficient": 0, "windowed": 1}
STAGE_HT, STAGE_WIENER = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-Wall", "-o", _LIB, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("pad0", C.c_int32),
        ("shape", C.c_int64 * MAXD),
        ("patch", C.c_int32 * MAXD), ("step", C.c_int32 * MAXD), ("search", C.c_int32 * MAXD),
        ("schedule", C.c_int32), ("passes", C.c_int32), ("shift_density", C.c_double),
        ("group_min", C.c_int32), ("group_max", C.c_int32),
        ("tau", C.c_double), ("gamma", C.c_double),
        ("spatial", C.c_int32), ("shrink", C.c_int32),
        ("lam", C.c_double), ("s_v", C.c_double), ("power_a", C.c_double),
        ("k_exact", C.c_int32), ("weight_model", C.c_int32), ("weight_scope", C.c_int32),
        ("mass_conservation", C.c_int32),
        ("kaiser_beta", C.c_double),
        ("noise_kind", C.c_int32), ("counts_integral", C.c_int32),
        ("sigma", C.c_double), ("s_p", C.c_double),
        ("metric", C.c_int32), ("policy", C.c_int32),
        ("match_t", C.c_double), ("struct_beta", C.c_double), ("struct_kappa", C.c_double),
        ("weight_domain", C.c_int32), ("pad1", C.c_int32),
        ("acov", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        P = C.POINTER(_Cfg)
        sig = {
            "orc_shift_list": (C.c_int, [i32, i32, d, vp, i32]),
            "orc_schedule": (i64, [P, vp, i64]),
            "orc_coverage": (C.c_int, [P, vp, vp]),
            "orc_haar_matrix": (C.c_int, [i32, vp]),
            "orc_spatial_matrices": (C.c_int, [i32, i32, vp, vp]),
            "orc_bior15_filters": (C.c_int, [vp, vp]),
            "orc_kaiser": (C.c_int, [i32, d, vp]),
            "orc_match": (C.c_int, [P, i32, vp, vp, vp, i64, vp, vp, vp, vp]),
            "orc_filter": (C.c_int, [P, i32, vp, vp, i64, vp, vp, vp, vp]),
            "orc_group_coeffs": (C.c_int, [P, i32, vp, vp, i32, vp, vp, vp, vp, vp]),
            "orc_aggregate": (C.c_int, [P, vp, i64, vp, vp, vp, vp, vp, vp]),
            "orc_run_stage": (C.c_int, [P, i32, vp, vp, vp]),
            "orc_denoise": (C.c_int, [P, P, vp, vp, vp]),
            "orc_phi": (d, [i32, d, d]),
            "orc_count_moments": (C.c_int, [i32, i32, vp, vp]),
            "orc_pair_score": (C.c_int, [i32, i32, d, d, d, i32, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


@dataclass
class Stage:
    """One stage's configuration (geometry, noise and profile)."""
    shape: Sequence[int]
    patch: Sequence[int]
    step: Sequence[int]
    search: Sequence[int]
    group_min: int = 2
    group_max: int = 16
    tau: float = -1.0           # < 0: c * P / 255^2 with c = 3000 (HT) / 400 (Wiener)
    gamma: float = 0.0
    spatial: str = "bior1.5"
    shrink: str = "hard"
    lam: float = 3.0
    s_v: float = 0.4
    power_a: float = 0.0
    k_exact: int = 0
    weight_model: str = "classic"
    weight_scope: str = "group"
    mass_conservation: bool = False
    kaiser_beta: float = 2.0
    schedule: str = "generated"
    shift_density: float = 2.0
    passes: int = 2
    noise: str = "poisson"
    counts_integral: bool = True
    metric: str = "ssd"         # HT matching distance (Poisson noise)
    policy: str = "fixed"       # acceptance calibration of a Poisson metric
    match_t: float = 3.0        # threshold multiplier t
    struct_beta: float = 0.1    # structural allowance beta_s (reference policy)
    struct_kappa: float = 1.0   # its intensity exponent kappa_s
    weight_domain: str = "coefficient"  # or "windowed" (synthesized domain)
    sigma: float = 0.0
    s_p: float = 1.0
    psd: Optional[np.ndarray] = None   # correlated noise: PSD on the array's DFT grid

    @property
    def P(self) -> int:
        return int(np.prod(self.patch))

    def cfg(self, stage: int) -> _Cfg:
        c = _Cfg()
        nd = len(self.shape)
        c.ndim = nd
        for d in range(nd):
            c.shape[d] = int(self.shape[d])
            c.patch[d] = int(self.patch[d])
            c.step[d] = int(self.step[d])
            c.search[d] = int(self.search[d])
        c.schedule = SCHED[self.schedule]
        c.passes = self.passes
        c.shift_density = self.shift_density
        c.group_min, c.group_max = self.group_min, self.group_max
        tau = self.tau
        if tau < 0:
            tau = (3000.0 if stage == STAGE_HT else 400.0) * self.P / 255.0 ** 2
        c.tau = tau
        c.gamma = self.gamma
        c.spatial = SPATIAL[self.spatial]
        c.shrink = SHRINK[self.shrink]
        c.lam, c.s_v, c.power_a = self.lam, self.s_v, self.power_a
        c.k_exact = self.k_exact
        c.weight_model = WMODEL[self.weight_model]
        c.weight_scope = WSCOPE[self.weight_scope]
        c.mass_conservation = int(bool(self.mass_conservation))
        c.kaiser_beta = self.kaiser_beta
        c.noise_kind = NOISE[self.noise]
        c.counts_integral = int(bool(self.counts_integral))
        c.sigma, c.s_p = self.sigma, self.s_p
        c.metric, c.policy = METRIC[self.metric], POLICY[self.policy]
        c.match_t, c.struct_beta, c.struct_kappa = self.match_t, self.struct_beta, self.struct_kappa
        c.weight_domain = WDOMAIN[self.weight_domain]
        if self.noise == "correlated":
            if self.psd is None:
                raise ValueError("correlated noise needs a power spectral density")
            acov = autocovariance(self.psd)
            if acov.shape != tuple(int(v) for v in self.shape):
                raise ValueError("the power spectral density must have the array's shape")
            c.acov = acov.ctypes.data
            c._keep = acov    # the C side reads it through the pointer
        return c


def autocovariance(psd: np.ndarray) -> np.ndarray:
    """Autocovariance c(tau) of stationary Gaussian noise from its power
    spectral density on the array's DFT grid (discrete Wiener-Khinchin
    relation, section Observation Models): c = ifftn(S) / |Omega|, real part
    (the autocovariance of a real field is real and even)."""
    S = np.asarray(psd, dtype=np.float64)
    return np.ascontiguousarray(np.real(np.fft.ifftn(S)) / S.size)


def plain_profile(shape, patch, step, search, s_p=1.0, group=(16, 32), mc=(False, False),
                  noise="poisson", sigma=0.0, counts_integral=True, psd=None):
    """The ablation reference levels ("plain"): SSD with gamma = 3 in the HT
    stage, no exact covariance planes, classic gain, classic group weights,
    hard threshold lambda = 3, s_v = 0.4, Kaiser beta = 2, generated (2, 2)."""
    common = dict(shape=tuple(shape), patch=tuple(patch), step=tuple(step), search=tuple(search),
                  noise=noise, s_p=s_p, sigma=sigma, counts_integral=counts_integral, psd=psd)
    ht = Stage(**common, group_max=group[0], gamma=3.0, spatial="bior1.5", shrink="hard",
               mass_conservation=mc[0])
    wie = Stage(**common, group_max=group[1], gamma=0.0, spatial="dct", shrink="wiener",
                mass_conservation=mc[1])
    return ht, wie


def standard_profile(shape, patch, step, search, s_p=1.0, group=(16, 32), mc=(False, False),
                     noise="poisson", sigma=0.0, counts_integral=True):
    """Appendix A standard profile: k = 4 exact covariance planes and variance /
    coefficient / patch weights in both stages (the Wiener gain mode is not
    stated there; the classic gain is kept)."""
    ht, wie = plain_profile(shape, patch, step, search, s_p, group, mc, noise, sigma,
                            counts_integral)
    ht = replace(ht, k_exact=4, weight_model="variance", weight_scope="patch")
    wie = replace(wie, k_exact=4, weight_model="variance", weight_scope="patch")
    return ht, wie


# ---------------------------------------------------------------- wrappers

def shift_list(j: int, h: int, rho: float) -> list:
    out = np.zeros(64, np.int32)
    n = lib().orc_shift_list(j, h, rho, _ptr(out), 64)
    _check(0 if n > 0 else n, "shift_list")
    return out[:n].tolist()


def schedule(st: Stage, stage: int = STAGE_HT) -> np.ndarray:
    c = st.cfg(stage)
    n = lib().orc_schedule(C.byref(c), None, 0)
    _check(0 if n >= 0 else int(n), "schedule")
    out = np.zeros(max(n, 1), np.int64)
    lib().orc_schedule(C.byref(c), _ptr(out), n)
    return out[:n]


def coverage(st: Stage, stage: int = STAGE_HT):
    """Coverage map C of the stage's schedule (array shape, uint32) and its
    (mean, standard deviation, CV): section Experiments, Shift Schedule
    Analysis."""
    c = st.cfg(stage)
    cov = np.zeros(tuple(int(v) for v in st.shape), np.uint32)
    stats = np.zeros(3)
    _check(lib().orc_coverage(C.byref(c), _ptr(cov), _ptr(stats)), "coverage")
    return cov, float(stats[0]), float(stats[1]), float(stats[2])


def haar(K: int) -> np.ndarray:
    H = np.zeros((K, K))
    _check(lib().orc_haar_matrix(K, _ptr(H)), "haar")
    return H


def spatial(kind: str, n: int):
    T = np.zeros((n, n))
    U = np.zeros((n, n))
    _check(lib().orc_spatial_matrices(SPATIAL[kind], n, _ptr(T), _ptr(U)), "spatial")
    return T, U


def bior15_filters():
    lo10 = np.zeros(10)
    lo2 = np.zeros(2)
    _check(lib().orc_bior15_filters(_ptr(lo10), _ptr(lo2)), "bior15")
    return lo10, lo2


def kaiser(n: int, beta: float) -> np.ndarray:
    w = np.zeros(n)
    _check(lib().orc_kaiser(n, beta, _ptr(w)), "kaiser")
    return w


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def match(st: Stage, stage: int, src, y, refs):
    c = st.cfg(stage)
    src = _f64(src).ravel()
    y = _f64(y).ravel()
    refs = np.ascontiguousarray(refs, dtype=np.int64)
    n = len(refs)
    g = st.group_max
    m = np.zeros((n, g), np.int32)
    cnt = np.zeros(n, np.int32)
    sc = np.zeros((n, g))
    acc = np.zeros(n, np.int32)
    _check(lib().orc_match(C.byref(c), stage, _ptr(src), _ptr(y), _ptr(refs), n, _ptr(m),
                           _ptr(cnt), _ptr(sc), _ptr(acc)), "match")
    return m, cnt, sc, acc


def phi(metric: str, r: float, c: float) -> float:
    """Per-entry contribution of a Poisson metric (eq. varphi)."""
    return lib().orc_phi(METRIC[metric], float(r), float(c))


def count_moments(metric: str, n: int):
    """Exact finite-count conditional mean and variance of phi given the
    pooled count n (Prop. universal finite-count moments)."""
    mu, v = C.c_double(), C.c_double()
    _check(lib().orc_count_moments(METRIC[metric], int(n), C.byref(mu), C.byref(v)), "moments")
    return mu.value, v.value


def pair_score(metric: str, policy: str, r, c, t=3.0, beta=0.1, kappa=1.0):
    """(score, threshold) of one reference / candidate pair of raw counts."""
    r = _f64(r).ravel()
    c = _f64(c).ravel()
    s, th = C.c_double(), C.c_double()
    _check(lib().orc_pair_score(METRIC[metric], POLICY[policy], t, beta, kappa, len(r), _ptr(r),
                                _ptr(c), C.byref(s), C.byref(th)), "pair_score")
    return s.value, th.value


def filter(st: Stage, stage: int, y, pilot, match_, count):
    c = st.cfg(stage)
    y = _f64(y).ravel()
    pil = None if pilot is None else _f64(pilot).ravel()
    match_ = np.ascontiguousarray(match_, dtype=np.int32)
    count = np.ascontiguousarray(count, dtype=np.int32)
    n = len(count)
    g = st.group_max
    patches = np.zeros((n, g, st.P))
    weights = np.zeros((n, g))
    _check(lib().orc_filter(C.byref(c), stage, _ptr(y), _ptr(pil), n, _ptr(match_),
                            _ptr(count), _ptr(patches), _ptr(weights)), "filter")
    return patches, weights


def group_coeffs(st: Stage, stage: int, y, pilot, origins):
    c = st.cfg(stage)
    y = _f64(y).ravel()
    pil = None if pilot is None else _f64(pilot).ravel()
    org = np.ascontiguousarray(origins, dtype=np.int32)
    K = len(org)
    Y = np.zeros((K, st.P))
    var = np.zeros((K, st.P))
    Cc = np.zeros((K, st.P))
    w = np.zeros(K)
    _check(lib().orc_group_coeffs(C.byref(c), stage, _ptr(y), _ptr(pil), K, _ptr(org),
                                  _ptr(Y), _ptr(var), _ptr(Cc), _ptr(w)), "group_coeffs")
    return Y, var, Cc, w


def aggregate(st: Stage, stage: int, y, match_, count, patches, weights, return_eta=False):
    c = st.cfg(stage)
    y = _f64(y).ravel()
    match_ = np.ascontiguousarray(match_, dtype=np.int32)
    count = np.ascontiguousarray(count, dtype=np.int32)
    patches = _f64(patches)
    weights = _f64(weights)
    out = np.zeros(int(np.prod(st.shape)))
    eta = np.zeros_like(out)
    _check(lib().orc_aggregate(C.byref(c), _ptr(y), len(count), _ptr(match_), _ptr(count),
                               _ptr(patches), _ptr(weights), _ptr(out), _ptr(eta)), "aggregate")
    out = out.reshape(tuple(st.shape))
    return (out, eta.reshape(tuple(st.shape))) if return_eta else out


def run_stage(st: Stage, stage: int, y, pilot=None) -> np.ndarray:
    c = st.cfg(stage)
    y = _f64(y).ravel()
    pil = None if pilot is None else _f64(pilot).ravel()
    out = np.zeros_like(y)
    _check(lib().orc_run_stage(C.byref(c), stage, _ptr(y), _ptr(pil), _ptr(out)), "run_stage")
    return out.reshape(tuple(st.shape))


def denoise(ht: Stage, wie: Stage, y):
    """Two-stage BMND; returns (pilot, output) in float64."""
    c1 = ht.cfg(STAGE_HT)
    c2 = wie.cfg(STAGE_WIENER)
    y = _f64(y).ravel()
    pilot = np.zeros_like(y)
    out = np.zeros_like(y)
    _check(lib().orc_denoise(C.byref(c1), C.byref(c2), _ptr(y), _ptr(pilot), _ptr(out)),
           "denoise")
    shp = tuple(ht.shape)
    return pilot.reshape(shp), out.reshape(shp)
