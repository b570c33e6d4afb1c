"""Python binding of the BMND MI355X library (``libbmnd.so``).

Argument marshalling only: every step of the denoising path runs in the
library's HIP kernels.  The C ABI is declared in ``include/bmnd.h``; the
functions below carry the same names and take torch tensors for device
buffers (their ``data_ptr()`` is passed) and the current torch stream.

The library is loaded on first use.  If it has not been built, a
``RuntimeError`` is raised: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmnd.so")

MAX_AXES = 8
OK, E_ARG, E_SHAPE, E_UNSUPPORTED, E_NOMEM, E_HIP, E_WORKSPACE, E_RANGE = 0, -1, -2, -3, -4, -5, -6, -7
E_BUDGET = -8
STAGE_HT, STAGE_WIENER = 0, 1
NOISE_GAUSSIAN, NOISE_POISSON, NOISE_CORRELATED = 0, 1, 2
SCHED = {"generated": 0, "balanced": 1, "sparse": 2, "off": 3}
SPATIAL = {"identity": 0, "dct": 1, "bior1.5": 2}
SHRINK = {"hard": 0, "soft": 1, "wiener": 2}
WEIGHT = {"classic": 0, "variance": 1, "risk": 2}
SCOPE = {"group": 0, "patch": 1}
PRESET_PLAIN, PRESET_STANDARD = 0, 1
METRIC_SSD, METRIC_DEVIANCE, METRIC_PEARSON, METRIC_ANSCOMBE = 0, 1, 2, 3
POLICY_FIXED, POLICY_REFERENCE, POLICY_STANDARDIZED = 0, 1, 2
MOMENT_MAX_COUNT = 4096
WDOMAIN_COEFFICIENT, WDOMAIN_WINDOWED = 0, 1


class BmndError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bmnd status {status}: {message}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("batch", C.c_int64),
                ("shape", C.c_int64 * MAX_AXES)]


class Noise(C.Structure):
    _fields_ = [("kind", C.c_int32), ("counts_integral", C.c_int32), ("sigma", C.c_double),
                ("s_p", C.c_double), ("d_corr", C.c_void_p)]


class StageParams(C.Structure):
    _fields_ = [
        ("patch", C.c_int32 * MAX_AXES), ("step", C.c_int32 * MAX_AXES),
        ("search", C.c_int32 * MAX_AXES),
        ("schedule", C.c_int32), ("passes", C.c_int32), ("shift_density", C.c_double),
        ("group_min", C.c_int32), ("group_max", C.c_int32),
        ("tau", C.c_double), ("gamma", C.c_double),
        ("spatial", C.c_int32), ("shrink", C.c_int32),
        ("lam", C.c_double), ("s_v", C.c_double), ("power_a", C.c_double),
        ("k_exact", C.c_int32), ("weight_model", C.c_int32), ("weight_scope", C.c_int32),
        ("mass_conservation", C.c_int32),
        ("kaiser_beta", C.c_double),
        ("match_metric", C.c_int32), ("match_policy", C.c_int32),
        ("match_t", C.c_double), ("struct_beta", C.c_double), ("struct_kappa", C.c_double),
        ("weight_domain", C.c_int32), ("reserved2", C.c_int32),
    ]


class Params(C.Structure):
    _fields_ = [("ht", StageParams), ("wiener", StageParams)]


class Job(C.Structure):
    """One entry of a batch (``bmnd_job``)."""
    _fields_ = [("d_y", C.c_void_p), ("d_out", C.c_void_p), ("d_pilot", C.c_void_p),
                ("geom", Geometry), ("noise", Noise), ("params", Params)]


BATCH_GRAPH = 1


EXPORTS = [
    "bmnd_last_error", "bmnd_version", "bmnd_params_default", "bmnd_reference_origins",
    "bmnd_reference_coverage",
    "bmnd_match_workspace_size", "bmnd_aggregate_workspace_size", "bmnd_workspace_size",
    "bmnd_match", "bmnd_filter", "bmnd_aggregate", "bmnd_denoise", "bmnd_stream_status",
    "bmnd_transform_matrices", "bmnd_haar_matrix", "bmnd_kaiser_window", "bmnd_count_moments",
    "bmnd_profile_begin", "bmnd_profile_end", "bmnd_batch_workspace_size", "bmnd_denoise_batch",
    "bmnd_correlated_size", "bmnd_correlated_prepare", "bmnd_denoise_noalloc",
    "bmnd_denoise_from_pilot", "bmnd_request_bytes", "bmnd_workspace_sums",
    "bmnd_cache_limits", "bmnd_autotune",
]
KERNEL_IDS = ["counts", "patch_sums", "match_ht", "match_wiener", "filter_ht", "filter_wiener",
              "zero", "normalize"]

_lib = None


def lib() -> C.CDLL:
    """Load libbmnd.so (built in-tree by ``paper_2609_34622_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2609_34622_amd.build` (no fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    G, N, S, PP = C.POINTER(Geometry), C.POINTER(Noise), C.POINTER(StageParams), C.POINTER(Params)
    sigs = {
        "bmnd_last_error": (C.c_char_p, []),
        "bmnd_version": (C.c_char_p, []),
        "bmnd_params_default": (i32, [i32, i32, PP]),
        "bmnd_reference_origins": (i32, [G, S, vp, i64, C.POINTER(i64)]),
        "bmnd_reference_coverage": (i32, [G, S, vp, vp]),
        "bmnd_match_workspace_size": (i32, [G, S, C.POINTER(sz)]),
        "bmnd_aggregate_workspace_size": (i32, [G, S, C.POINTER(sz)]),
        "bmnd_workspace_size": (i32, [G, N, PP, C.POINTER(sz)]),
        "bmnd_match": (i32, [i32, vp, G, N, S, vp, i64, vp, vp, vp, vp, sz, vp]),
        "bmnd_filter": (i32, [i32, vp, vp, G, N, S, i64, vp, vp, vp, vp, vp]),
        "bmnd_aggregate": (i32, [vp, G, S, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
        "bmnd_denoise": (i32, [vp, G, N, PP, vp, vp, vp, sz, vp]),
        "bmnd_stream_status": (i32, [vp]),
        "bmnd_transform_matrices": (i32, [i32, i32, vp, vp]),
        "bmnd_haar_matrix": (i32, [i32, vp]),
        "bmnd_kaiser_window": (i32, [i32, C.c_double, vp]),
        "bmnd_count_moments": (i32, [i32, i32, vp, vp]),
        "bmnd_profile_begin": (i32, []),
        "bmnd_profile_end": (i32, [vp, vp, i32]),
        "bmnd_batch_workspace_size": (i32, [i32, C.POINTER(Job), C.POINTER(sz)]),
        "bmnd_denoise_batch": (i32, [i32, C.POINTER(Job), vp, sz, i32, vp]),
        "bmnd_correlated_size": (i32, [G, PP, C.POINTER(sz)]),
        "bmnd_correlated_prepare": (i32, [vp, G, PP, vp, sz, vp]),
        "bmnd_denoise_noalloc": (i32, [vp, G, N, PP, vp, vp, vp]),
        "bmnd_denoise_from_pilot": (i32, [vp, vp, G, N, PP, vp, vp, sz, vp]),
        "bmnd_request_bytes": (i32, [G, N, PP, sz, C.POINTER(sz)]),
        "bmnd_workspace_sums": (i32, [G, N, PP, C.POINTER(sz), C.POINTER(sz)]),
        "bmnd_cache_limits": (i32, [sz, sz]),
        "bmnd_autotune": (i32, [vp, G, N, PP, vp, vp, sz, vp, C.POINTER(i32), vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise BmndError(status, lib().bmnd_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch

    return int(torch.cuda.current_stream().cuda_stream)


def _require(t, dtype, numel: Optional[int] = None, name: str = "tensor"):
    import torch

    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    del torch


# ------------------------------------------------------------------ structs

def geometry(shape: Sequence[int], batch: int = 1) -> Geometry:
    g = Geometry()
    g.ndim = len(shape)
    g.batch = int(batch)
    for d, v in enumerate(shape):
        g.shape[d] = int(v)
    return g


def poisson(s_p: float, counts_integral: bool = True) -> Noise:
    n = Noise()
    n.kind = NOISE_POISSON
    n.counts_integral = int(bool(counts_integral))
    n.s_p = float(s_p)
    return n


def gaussian(sigma: float) -> Noise:
    n = Noise()
    n.kind = NOISE_GAUSSIAN
    n.sigma = float(sigma)
    return n


def correlated(tables) -> Noise:
    """Stationary correlated Gaussian noise described by the device tables
    that ``bmnd_correlated_prepare`` wrote (the Noise keeps them alive)."""
    n = Noise()
    n.kind = NOISE_CORRELATED
    n.d_corr = _ptr(tables)
    n._keep = tables
    return n


def set_axes(sp: StageParams, patch=None, step=None, search=None):
    for name, vals in (("patch", patch), ("step", step), ("search", search)):
        if vals is not None:
            arr = getattr(sp, name)
            for d, v in enumerate(vals):
                arr[d] = int(v)
    return sp


# ------------------------------------------------------------- C ABI calls

def bmnd_version() -> str:
    return lib().bmnd_version().decode()


def bmnd_params_default(preset: int, ndim: int) -> Params:
    p = Params()
    _check(lib().bmnd_params_default(preset, ndim, C.byref(p)))
    return p


def bmnd_reference_coverage(geom: Geometry, sp: StageParams):
    """Coverage map C of the stage's reference schedule (uint32, the array's
    shape) and (mean, standard deviation, CV) of C."""
    shape = tuple(int(geom.shape[d]) for d in range(geom.ndim))
    cov = np.zeros(shape, np.uint32)
    stats = np.zeros(3)
    _check(lib().bmnd_reference_coverage(C.byref(geom), C.byref(sp), cov.ctypes.data,
                                         stats.ctypes.data))
    return cov, float(stats[0]), float(stats[1]), float(stats[2])


def bmnd_reference_origins(geom: Geometry, sp: StageParams) -> np.ndarray:
    n = C.c_int64(0)
    _check(lib().bmnd_reference_origins(C.byref(geom), C.byref(sp), None, 0, C.byref(n)))
    out = np.zeros(max(n.value, 1), np.int64)
    _check(lib().bmnd_reference_origins(C.byref(geom), C.byref(sp), out.ctypes.data, n.value,
                                        C.byref(n)))
    return out[: n.value]


def bmnd_transform_matrices(spatial: str, n: int):
    T = np.zeros((n, n))
    U = np.zeros((n, n))
    _check(lib().bmnd_transform_matrices(SPATIAL[spatial], n, T.ctypes.data, U.ctypes.data))
    return T, U


def bmnd_haar_matrix(K: int) -> np.ndarray:
    H = np.zeros((K, K))
    _check(lib().bmnd_haar_matrix(K, H.ctypes.data))
    return H


def bmnd_kaiser_window(n: int, beta: float) -> np.ndarray:
    w = np.zeros(n)
    _check(lib().bmnd_kaiser_window(n, beta, w.ctypes.data))
    return w


def bmnd_count_moments(metric: int, nmax: int):
    """The library's finite-count moment tables mu[0..nmax], v[0..nmax]."""
    mu = np.zeros(nmax + 1)
    v = np.zeros(nmax + 1)
    _check(lib().bmnd_count_moments(metric, nmax, mu.ctypes.data, v.ctypes.data))
    return mu, v


def bmnd_correlated_size(geom: Geometry, params: Params) -> int:
    b = C.c_size_t(0)
    _check(lib().bmnd_correlated_size(C.byref(geom), C.byref(params), C.byref(b)))
    return b.value


def bmnd_correlated_prepare(psd, geom: Geometry, params: Params, tables=None, stream=None):
    """Tables of stationary correlated Gaussian noise from its power spectral
    density ``psd`` (device float64, the array's shape, C-order); returns
    the uint8 device tensor that holds them (``tables`` if given)."""
    import torch

    n = bmnd_correlated_size(geom, params)
    _require(psd, torch.float64, int(np.prod([geom.shape[d] for d in range(geom.ndim)])), "psd")
    if tables is None:
        tables = torch.empty(n, dtype=torch.uint8, device=psd.device)
    _require(tables, torch.uint8, n, "tables")
    _check(lib().bmnd_correlated_prepare(_ptr(psd), C.byref(geom), C.byref(params), _ptr(tables),
                                         tables.numel(), _stream(stream)))
    return tables


def bmnd_match_workspace_size(geom: Geometry, sp: StageParams) -> int:
    b = C.c_size_t(0)
    _check(lib().bmnd_match_workspace_size(C.byref(geom), C.byref(sp), C.byref(b)))
    return b.value


def bmnd_aggregate_workspace_size(geom: Geometry, sp: StageParams) -> int:
    b = C.c_size_t(0)
    _check(lib().bmnd_aggregate_workspace_size(C.byref(geom), C.byref(sp), C.byref(b)))
    return b.value


BLOCK_RULES = 6


def bmnd_autotune(y, geom, noise, params, out, ws, stream=None):
    """Time the candidate block rules of the 2-D / 3-D kernels on this input
    and keep the fastest for its shape and parameters; returns (chosen rule
    or -1, per-rule milliseconds)."""
    import torch

    _require(y, torch.float32, name="y")
    _require(out, torch.float32, name="out")
    ch = C.c_int32(-1)
    ms = np.zeros(BLOCK_RULES)
    _check(lib().bmnd_autotune(_ptr(y), C.byref(geom), C.byref(noise), C.byref(params), _ptr(out),
                               _ptr(ws), ws.numel() * ws.element_size(), _stream(stream),
                               C.byref(ch), ms.ctypes.data))
    return ch.value, ms.tolist()


def bmnd_cache_limits(host_bytes: int = 0, device_bytes: int = 0) -> None:
    """Byte budgets of the per-shape schedule caches (0: the default)."""
    _check(lib().bmnd_cache_limits(host_bytes, device_bytes))


def bmnd_workspace_sums(geom: Geometry, noise: Noise, params: Params):
    """(numerator offset, denominator offset): bytes into a bmnd_denoise
    workspace where the last stage's FP64 sums stay after the call."""
    a, b = C.c_size_t(0), C.c_size_t(0)
    _check(lib().bmnd_workspace_sums(C.byref(geom), C.byref(noise), C.byref(params), C.byref(a),
                                     C.byref(b)))
    return a.value, b.value


def bmnd_request_bytes(geom: Geometry, noise: Noise, params: Params, budget: int = 0) -> int:
    """Device bytes a denoise request holds (arrays and workspace); raises
    BmndError(E_BUDGET) when budget > 0 and the request exceeds it."""
    b = C.c_size_t(0)
    _check(lib().bmnd_request_bytes(C.byref(geom), C.byref(noise), C.byref(params), budget,
                                    C.byref(b)))
    return b.value


def bmnd_workspace_size(geom: Geometry, noise: Noise, params: Params) -> int:
    b = C.c_size_t(0)
    _check(lib().bmnd_workspace_size(C.byref(geom), C.byref(noise), C.byref(params), C.byref(b)))
    return b.value


def bmnd_match(stage, src, geom, noise, sp, refs, match, count, ws, stream=None, score=None):
    """Block matching of the given references; `score` (float32, the shape
    of `match`, optional) receives each member's distance to its reference
    in the units of tau (0 for the reference and beyond the group size)."""
    import torch

    _require(src, torch.float32, name="src")
    _require(refs, torch.int64, name="refs")
    _require(match, torch.int32, name="match")
    _require(count, torch.int32, name="count")
    if score is not None:
        _require(score, torch.float32, name="score")
        if score.numel() != match.numel():
            raise ValueError("score must have as many entries as match")
    n_refs = int(refs.numel())
    _check(lib().bmnd_match(stage, _ptr(src), C.byref(geom), C.byref(noise), C.byref(sp),
                            _ptr(refs), n_refs, _ptr(match), _ptr(count), _ptr(score), _ptr(ws),
                            0 if ws is None else ws.numel() * ws.element_size(), _stream(stream)))


def bmnd_filter(stage, y, pilot, geom, noise, sp, n_refs, match, count, patches, weights,
                stream=None):
    import torch

    for t, nm in ((y, "y"), (pilot, "pilot"), (patches, "patches"), (weights, "weights")):
        _require(t, torch.float32, name=nm)
    _check(lib().bmnd_filter(stage, _ptr(y), _ptr(pilot), C.byref(geom), C.byref(noise),
                             C.byref(sp), int(n_refs), _ptr(match), _ptr(count), _ptr(patches),
                             _ptr(weights), _stream(stream)))


def bmnd_aggregate(y, geom, sp, n_refs, match, count, patches, weights, out, ws, stream=None):
    _check(lib().bmnd_aggregate(_ptr(y), C.byref(geom), C.byref(sp), int(n_refs), _ptr(match),
                                _ptr(count), _ptr(patches), _ptr(weights), _ptr(out), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def bmnd_denoise(y, geom, noise, params, out, pilot, ws, stream=None):
    import torch

    _require(y, torch.float32, name="y")
    _require(out, torch.float32, name="out")
    _require(pilot, torch.float32, name="pilot")
    _check(lib().bmnd_denoise(_ptr(y), C.byref(geom), C.byref(noise), C.byref(params), _ptr(out),
                              _ptr(pilot), _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))


def bmnd_denoise_from_pilot(y, pilot, geom, noise, params, out, ws, stream=None):
    """The Wiener stage of bmnd_denoise from a supplied pilot."""
    import torch

    for t, nm in ((y, "y"), (pilot, "pilot"), (out, "out")):
        _require(t, torch.float32, name=nm)
    _check(lib().bmnd_denoise_from_pilot(_ptr(y), _ptr(pilot), C.byref(geom), C.byref(noise),
                                         C.byref(params), _ptr(out), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def bmnd_denoise_noalloc(y, geom, noise, params, out, pilot=None, stream=None):
    """bmnd_denoise with all device scratch in the library's static array
    (no workspace argument, no device allocation by the library)."""
    import torch

    _require(y, torch.float32, name="y")
    _require(out, torch.float32, name="out")
    _require(pilot, torch.float32, name="pilot")
    _check(lib().bmnd_denoise_noalloc(_ptr(y), C.byref(geom), C.byref(noise), C.byref(params),
                                      _ptr(out), _ptr(pilot), _stream(stream)))


def bmnd_profile_begin():
    _check(lib().bmnd_profile_begin())


def bmnd_profile_end() -> dict:
    """Stop tracing; returns {kernel: (total_ms, launches)}."""
    n = len(KERNEL_IDS)
    ms = np.zeros(n)
    cnt = np.zeros(n, np.int64)
    _check(lib().bmnd_profile_end(ms.ctypes.data, cnt.ctypes.data, n))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_IDS)}


def bmnd_stream_status(stream=None):
    _check(lib().bmnd_stream_status(_stream(stream)))


# -------------------------------------------------------------- convenience

def denoise(y, noise: Noise, params: Optional[Params] = None, batched: bool = False,
            return_pilot: bool = False):
    """Two-stage BMND of a float32 device tensor.  With ``batched`` the
    leading axis indexes independent arrays.  Returns the output tensor (and
    the pilot).  Allocates the output, pilot and workspace with torch."""
    import torch

    shape = tuple(y.shape[1:]) if batched else tuple(y.shape)
    batch = y.shape[0] if batched else 1
    geom = geometry(shape, batch)
    if params is None:
        params = bmnd_params_default(PRESET_PLAIN, len(shape))
    ws = torch.empty(bmnd_workspace_size(geom, noise, params), dtype=torch.uint8, device=y.device)
    out = torch.empty_like(y)
    pilot = torch.empty_like(y)
    bmnd_denoise(y.contiguous(), geom, noise, params, out, pilot, ws)
    return (out, pilot) if return_pilot else out


def make_jobs(entries) -> "C.Array":
    """A ``bmnd_job`` table from (y, out, pilot_or_None, geom, noise, params)
    tuples of device tensors and parameter structs."""
    import torch

    arr = (Job * len(entries))()
    for i, (y, out, pilot, geom, noise, params) in enumerate(entries):
        _require(y, torch.float32, name="y")
        _require(out, torch.float32, name="out")
        _require(pilot, torch.float32, name="pilot")
        arr[i].d_y, arr[i].d_out, arr[i].d_pilot = _ptr(y), _ptr(out), _ptr(pilot)
        arr[i].geom, arr[i].noise, arr[i].params = geom, noise, params
    return arr


def bmnd_batch_workspace_size(jobs) -> int:
    n = C.c_size_t(0)
    _check(lib().bmnd_batch_workspace_size(len(jobs), jobs, C.byref(n)))
    return n.value


def bmnd_denoise_batch(jobs, ws, flags: int = 0, stream=None):
    _check(lib().bmnd_denoise_batch(len(jobs), jobs, _ptr(ws), ws.numel() * ws.element_size(),
                                    int(flags), _stream(stream)))
