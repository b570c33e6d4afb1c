#!/usr/bin/env python3
"""Throughput of the two-stage BMND hot path on one MI355X.

Workload (default): the 3-D phantom batch -- 4 low-count volumes of
256 x 256 x 128 (nested ellipsoids on a smooth background, each with its own
peak and so its own Poisson scale s_P = 1 / peak), patch 4 x 4 x 4, step 3,
search window 11^3, groups 16 / 32, plain profile, aggregation-aware mass
conservation in both stages.  One step is one complete two-stage denoise of
every volume (matching, filtering, aggregation and mass conservation of both
stages), one library call per volume with that volume's noise model, inputs
resident in HBM.  The 1-D ECG batch and the 2-D microscopy stack are timed
the same way after it (shorter runs), each with its own roofline.

Prints one JSON line: metric, value (denoised Mvox/s), roofline of the
dominant kernel (HIP events on the launch stream during the timed region),
the FP64 oracle timed on the host cores on a bounded sample (crops of the
same arrays), and the GPU's maximum relative error against that oracle on
the same sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # published FP32 vector peak (packed; dense FP32 matrix alike)
PEAK_INT32_TOPS = 78.6       # 32-bit integer VALU, multiply-add counted as 2:
                             # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2
PEAK_DOT4_TOPS = 314.6       # v_dot4_u32_u8: 4 multiply-adds per lane per instruction
PEAK_HBM_GBS = 8000.0
COPY_KERNEL_HINT = "MulFunctor"   # the calibration kernel: dst = src * 1
METRIC = "denoised Mvox/s (both stages) at \u22641e-4 rel err; serving p50/p99 latency"
REL_ERR_BAR = 1e-4
AUTOTUNE = True

WORKLOADS = {
    "ecg-1d-batch": dict(shape=(65536,), batch=256, patch=(32,), step=(4,), search=(256,),
                         group=(16, 16), mc=(False, False)),
    "image-2d-128": dict(shape=(128, 128), batch=1, patch=(8, 8), step=(3, 3), search=(39, 39),
                         group=(16, 32), mc=(False, False)),
    "microscopy-2d-16x1024": dict(shape=(1024, 1024), batch=16, patch=(8, 8), step=(3, 3),
                                  search=(39, 39), group=(16, 32), mc=(False, False)),
    "phantom-3d-4x256x256x128": dict(shape=(256, 256, 128), batch=4, patch=(4, 4, 4),
                                     step=(3, 3, 3), search=(11, 11, 11), group=(16, 32),
                                     mc=(True, True)),
}
# bounded oracle sample per workload: (arrays, crop shape or None for whole arrays)
CPU_SAMPLE = {
    "ecg-1d-batch": (8, None),
    "image-2d-128": (1, None),
    "microscopy-2d-16x1024": (4, (128, 128)),
    "phantom-3d-4x256x256x128": (4, (48, 48, 48)),
}


def make_input(name: str, w: dict):
    """The workload's arrays and their Poisson scales: (y [batch, *shape]
    float32, s_p list).  Every array keeps its own s_P (Def. scaled-Poisson
    observation model); the ECG signals share one by construction."""
    from paper_2609_34622_amd import synth

    if name == "ecg-1d-batch":
        s = synth.ecg_batch(n_signals=w["batch"], length=w["shape"][0], seed=2000)
        return np.ascontiguousarray(s.y, np.float32), [s.s_p] * w["batch"]
    if name == "image-2d-128":
        s = synth.image_2d_small(1000)
        return s.y[None].astype(np.float32), [s.s_p]
    ys, sps = [], []
    for b in range(w["batch"]):
        if name.startswith("microscopy"):
            s = synth.microscopy_2d(seed=3000 + b, size=w["shape"][0])
        else:
            s = synth.phantom_3d(seed=4000 + b, shape=w["shape"])
        ys.append(s.y)
        sps.append(s.s_p)
    return np.ascontiguousarray(np.stack(ys), np.float32), sps


def crops(name: str, y: np.ndarray, sps):
    """The bounded sample the oracle denoises: whole arrays, or a centred
    crop of each of the first arrays (with that array's s_P)."""
    n, shape = CPU_SAMPLE[name]
    out = []
    for b in range(min(n, y.shape[0])):
        a = y[b]
        if shape is not None:
            sl = tuple(slice((a.shape[d] - shape[d]) // 2, (a.shape[d] - shape[d]) // 2 + shape[d])
                       for d in range(a.ndim))
            a = a[sl]
        out.append((np.ascontiguousarray(a), sps[b]))
    return out


def _oracle_one(args):
    name, a, s_p = args
    import oracle as O

    w = WORKLOADS[name]
    ht, wie = O.plain_profile(a.shape, w["patch"], w["step"], w["search"], s_p=s_p,
                              group=w["group"], mc=w["mc"])
    t0 = time.perf_counter()
    pil, out = O.denoise(ht, wie, a)
    return (pil, out), time.perf_counter() - t0


def cpu_baseline(name: str, sample):
    """The oracle (FP64, single-threaded C) on the bounded sample: once on one
    core, then one process per host core (up to 16) over the sample repeated,
    for the all-core figure.  Runs before the GPU is touched (the worker
    processes are forked)."""
    import multiprocessing as mp
    import platform
    import subprocess

    outs, t1 = [], 0.0
    for a, s_p in sample:
        o, dt = _oracle_one((name, a, s_p))
        outs.append(o)
        t1 += dt
    vox = sum(a.size for a, _ in sample)
    ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    jobs = [(name, *sample[i % len(sample)]) for i in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_one, jobs)
    wall = time.perf_counter() - t0
    model = platform.processor() or ""
    try:
        for ln in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if ln.startswith("Model name"):
                model = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    shp = CPU_SAMPLE[name][1]
    what = (f"{len(sample)} arrays" if shp is None else
            f"{len(sample)} centred {'x'.join(map(str, shp))} crops (one per array, own s_P)")
    return outs, {
        "value": round(sum(j[1].size for j in jobs) / wall / 1e6, 5), "unit": "Mvox/s",
        "cores": workers, "kind": "oracle",
        "sample": f"{what} of the same workload, both stages; all-core: {workers} processes, "
                  f"one array each, {wall:.1f} s wall",
        "single_core": {"value": round(vox / t1 / 1e6, 5), "seconds": round(t1, 2)},
        "nproc": ncpu, "cpu_model": model}


def candidates_per_ref(shape, patch, search, refs):
    """Number of non-reference candidates of each reference (clipped window)."""
    coords = np.stack(np.unravel_index(refs, shape), axis=1)
    n = np.ones(len(refs), np.int64)
    for d in range(len(shape)):
        ell = shape[d] - patch[d]
        lo = np.maximum(coords[:, d] - search[d] // 2, 0)
        hi = np.minimum(coords[:, d] + search[d] - 1 - search[d] // 2, ell)
        n *= hi - lo + 1
    return n - 1


# kernel names of the library's kernels in rocprofv3 output, by stage (a
# stage may run two kernels: byte-count matching and its record fallback;
# the N-D filter runs two sweeps under mass conservation).  The window
# convolution that turns per-origin weights into the denominator runs once in
# each N-D filter stage; its counters are added to both filter stages.
KERNEL_SYMBOLS = {
    "filter_ht": [r"k_filter_1d<[01],", r"k_filter_nd<\d+,\d+,\d+,[01],"],
    "filter_wiener": [r"k_filter_1d<2,", r"k_filter_nd<\d+,\d+,\d+,2,"],
    "match_ht": [r"k_match_1d_u8<", r"k_match_1d_rec<", r"k_match_1d_f<2,", r"k_match_nd<0,",
                 r"k_match_blk<0,"],
    "match_wiener": [r"k_match_1d_f<3,", r"k_match_nd<3,", r"k_match_blk<3,"],
    "window_conv": [r"k_window_conv(_tiled)?<"],
}


def kernel_label(kname: str):
    import re

    flat = kname.replace(" ", "")
    for k, pats in KERNEL_SYMBOLS.items():
        if any(re.search(pat, flat) for pat in pats):
            return k
    return None


TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def _kernel_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_34622_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def summarize_pmc(dbs, copy_mib: int):
    """Per-launch FETCH_SIZE / WRITE_SIZE (KiB) of the library kernels and of
    the calibration copy, scaled to bytes by the copy's known traffic."""
    import sqlite3

    vals = {}
    copy_bytes = None
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, counter_name, sum(value), count(distinct dispatch_id) "
                           "from counters_collection group by kernel_name, counter_name").fetchall()
        grid = con.execute("select kernel_name, max(grid_size) from counters_collection "
                           "group by kernel_name").fetchall()
        grid = dict(grid)
        for kname, cname, total, ndisp in rows:
            key = kernel_label(kname)
            if key is None and COPY_KERNEL_HINT in kname and grid.get(kname, 0) > (1 << 20):
                key = "copy"
            if key is None:
                continue
            # per launch of the stage: the stage's kernels summed
            d = vals.setdefault(key, {})
            d[cname] = d.get(cname, 0.0) + float(total) / max(int(ndisp), 1)
    out = {"kernel_sources": _kernel_sources_digest(), "copy_probe_mib": copy_mib, "kernels": {}}
    cp = vals.get("copy", {})
    out["copy_probe_kib"] = cp
    conv = vals.get("window_conv", {})
    for k, v in vals.items():
        if k == "copy":
            continue
        e = {"fetch_kib": v.get("FETCH_SIZE"), "write_kib": v.get("WRITE_SIZE")}
        if k.startswith("filter") and conv:
            # one window convolution per N-D filter stage launch
            e = {"fetch_kib": e["fetch_kib"] + conv.get("FETCH_SIZE", 0.0),
                 "write_kib": e["write_kib"] + conv.get("WRITE_SIZE", 0.0),
                 "includes_window_conv": True}
        out["kernels"][k] = e
    out["note"] = ("scale: bytes = KiB * 1024 * (copy bytes / copy KiB*1024) per counter; "
                   "copy bytes = --copy-probe-mib MiB read and written")
    return out


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if absent or taken on other kernel sources."""
    path = os.path.join(TRAFFIC_DIR, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources") != _kernel_sources_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    cp = t.get("copy_probe_kib", {})
    mib = t.get("copy_probe_mib")
    if not k or not cp or not mib or not cp.get("FETCH_SIZE") or not cp.get("WRITE_SIZE"):
        return None
    nbytes = mib * (1 << 20)
    f_scale = nbytes / (cp["FETCH_SIZE"] * 1024.0)
    w_scale = nbytes / (cp["WRITE_SIZE"] * 1024.0)
    return round(k["fetch_kib"] * 1024.0 * f_scale + k["write_kib"] * 1024.0 * w_scale)


def _mixed_arrays(seed: int, n_each: int, len_1d, side_2d, side_3d):
    """Uneven arrays for the batched comparison: n_each 1-D signals, 2-D
    images and 3-D volumes of log-uniform sizes, as in the serving trace."""
    from paper_2609_34622_amd import serving

    return serving.make_trace(3 * n_each, 1.0, seed, len_1d=len_1d, side_2d=side_2d,
                              side_3d=side_3d, mix=(1, 1, 1))


def bench_batched(B, torch, reps: int = 3) -> dict:
    """The plain per-array path (one bmnd_denoise after another on one stream)
    against bmnd_denoise_batch (concurrent streams, replayed graph) on the
    same device-resident mixed arrays."""
    from paper_2609_34622_amd import serving

    reqs = _mixed_arrays(6000, 8, (16384, 65536), (128, 384), (32, 56))
    ys = [torch.from_numpy(r.y).cuda() for r in reqs]
    outs = [torch.empty_like(y) for y in ys]
    geoms = [B.geometry(r.y.shape) for r in reqs]
    noises = [B.poisson(r.s_p) for r in reqs]
    wss = [torch.empty(serving.request_bytes(r) - 2 * r.y.nbytes, dtype=torch.uint8, device="cuda")
           for r in reqs]
    jobs = B.make_jobs([(ys[i], outs[i], None, geoms[i], noises[i], reqs[i].params)
                        for i in range(len(reqs))])
    bws = torch.empty(B.bmnd_batch_workspace_size(jobs), dtype=torch.uint8, device="cuda")
    vox = sum(r.voxels for r in reqs)

    def plain():
        for i in range(len(reqs)):
            B.bmnd_denoise(ys[i], geoms[i], noises[i], reqs[i].params, outs[i], None, wss[i])

    def batched():
        B.bmnd_denoise_batch(jobs, bws, flags=B.BATCH_GRAPH)

    res = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"mvox_per_s": round(vox / dt / 1e6, 3), "ms": round(dt * 1e3, 3)}
    B.bmnd_stream_status()
    return {"arrays": len(reqs), "voxels": vox,
            "mix": "8 1-D (16k-64k samples), 8 2-D (128^2-384^2), 8 3-D (32^3-56^3, mass "
                   "conservation), seeded log-uniform sizes; device-resident",
            "plain": res["plain"], "batched": res["batched"],
            "speedup": round(res["plain"]["ms"] / res["batched"]["ms"], 3)}


def bench_serving(B, torch, n: int = 2000) -> dict:
    """Continuous batching against the plain one-at-a-time path on one seeded
    trace of `n` mixed requests (host arrays in, host results out): 40 %
    1-D signals of 8k-256k samples, 40 % 2-D images of 256^2-2048^2, 20 %
    3-D volumes of 64^3-256^3 (mass conservation), peaks log-uniform in
    [2, 100].  Four passes over the same requests: both paths with every
    request arriving at 0 (saturating; the plain path's pass also fills the
    library's per-shape caches and gives its capacity), then both at
    seeded Poisson arrivals at 0.7 of that capacity."""
    from paper_2609_34622_amd import serving

    t0 = time.perf_counter()
    trace = serving.make_trace_crops(n, 7001, torch)
    gen_s = time.perf_counter() - t0
    vox = sum(r.voxels for r in trace)
    kinds = [sum(1 for r in trace if r.y.ndim == d) for d in (1, 2, 3)]
    print(f"serving trace: {n} requests, {vox / 1e9:.3f} G voxels, generated in {gen_s:.1f} s",
          file=sys.stderr, flush=True)
    budget = 64 << 30

    def clear():
        for r in trace:
            r.out = None

    def rnd(d):
        return {k: round(v, 3) for k, v in d.items()}

    serving.set_rate(trace, float("inf"))
    fifo_sat = serving.serve_fifo(trace)
    clear()
    print(f"serving: plain path saturated {fifo_sat['mvox_per_s']:.1f} Mvox/s",
          file=sys.stderr, flush=True)
    srv = serving.Server(budget_bytes=budget, slots=4)
    cont_sat = srv.run(trace)
    clear()
    print(f"serving: continuous saturated {cont_sat['mvox_per_s']:.1f} Mvox/s",
          file=sys.stderr, flush=True)
    rate = 0.7 * fifo_sat["requests"] / fifo_sat["makespan_s"]
    serving.set_rate(trace, rate)
    cont = srv.run(trace)
    clear()
    fifo = serving.serve_fifo(trace)
    clear()
    print(f"serving: at {rate:.2f} req/s continuous p99 {cont['p99_ms']:.1f} ms, plain p99 "
          f"{fifo['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    return {"requests": n, "voxels": vox, "kinds_1d_2d_3d": kinds,
            "arrival_rate_per_s": round(rate, 3), "hbm_budget_gib": budget >> 30,
            "trace": "seeded; 40% 1-D (8k-256k samples), 40% 2-D (256^2-2048^2), 20% 3-D "
                     "(64^3-256^3, mass conservation); crops of full-size ECG, microscopy, "
                     "disc/rectangle and phantom means rescaled to peaks log-uniform in [2, 100], "
                     "Poisson-sampled with a seeded device generator",
            "admission": "4 streams, HBM budget (bmnd_request_bytes), in-flight work at most "
                         "half the largest request seen so far",
            "generation_s": round(gen_s, 1),
            "saturating": {"continuous": rnd(cont_sat), "plain_fifo": rnd(fifo_sat),
                           "speedup": round(cont_sat["mvox_per_s"] / fifo_sat["mvox_per_s"], 3)},
            "fixed_rate": {"continuous": rnd(cont), "plain_fifo": rnd(fifo)}}


def bench_standard(B, torch, workload: str = "image-2d-128", reps: int = 10) -> dict:
    """The standard profile (exact shared-source planes k_ex = 4, variance
    weights in patch scope) beside the plain profile on the same
    device-resident input."""
    w = WORKLOADS[workload]
    y_np, sps = make_input(workload, w)
    s_p = sps[0]
    shape, batch = w["shape"], w["batch"]
    y = torch.from_numpy(np.ascontiguousarray(y_np)).cuda()
    geom = B.geometry(shape, batch)
    noise = B.poisson(s_p)
    res = {}
    for name, preset in (("plain", B.PRESET_PLAIN), ("standard", B.PRESET_STANDARD)):
        p = B.bmnd_params_default(preset, len(shape))
        for sp in (p.ht, p.wiener):
            B.set_axes(sp, patch=w["patch"], step=w["step"], search=w["search"])
        p.ht.group_max, p.wiener.group_max = w["group"]
        p.ht.mass_conservation, p.wiener.mass_conservation = map(int, w["mc"])
        ws = torch.empty(B.bmnd_workspace_size(geom, noise, p), dtype=torch.uint8, device="cuda")
        out = torch.empty_like(y)
        B.bmnd_denoise(y, geom, noise, p, out, None, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.bmnd_denoise(y, geom, noise, p, out, None, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"mvox_per_s": round(batch * int(np.prod(shape)) / dt / 1e6, 3),
                     "ms": round(dt * 1e3, 3), "k_exact": int(p.ht.k_exact)}
        del ws, out
    B.bmnd_stream_status()
    return {"workload": workload, **res}


def bench_poisson_metrics(B, torch, n_signals: int = 16, reps: int = 3) -> dict:
    """HT matching with the Poisson-likelihood metrics (deviance, Pearson,
    Anscombe-SSD; fixed and candidate-standardized policies) beside SSD on
    ECG signals of the headline workload's shape (fewer of them)."""
    from paper_2609_34622_amd import synth

    w = WORKLOADS["ecg-1d-batch"]
    s = synth.ecg_batch(n_signals=n_signals, length=w["shape"][0], seed=2000)
    shape = w["shape"]
    y = torch.from_numpy(np.ascontiguousarray(s.y, np.float32)).cuda()
    geom = B.geometry(shape, n_signals)
    noise = B.poisson(s.s_p)
    res = {}
    for name, metric, policy in (("ssd", B.METRIC_SSD, B.POLICY_FIXED),
                                 ("deviance", B.METRIC_DEVIANCE, B.POLICY_FIXED),
                                 ("deviance_standardized", B.METRIC_DEVIANCE, B.POLICY_STANDARDIZED),
                                 ("pearson_standardized", B.METRIC_PEARSON, B.POLICY_STANDARDIZED),
                                 ("anscombe_reference", B.METRIC_ANSCOMBE, B.POLICY_REFERENCE)):
        p = B.bmnd_params_default(B.PRESET_PLAIN, 1)
        B.set_axes(p.ht, patch=w["patch"], step=w["step"], search=w["search"])
        p.ht.group_max = w["group"][0]
        p.ht.match_metric, p.ht.match_policy = metric, policy
        refs = B.bmnd_reference_origins(B.geometry(shape), p.ht)
        m = torch.empty((n_signals, len(refs), p.ht.group_max), dtype=torch.int32, device="cuda")
        c = torch.empty((n_signals, len(refs)), dtype=torch.int32, device="cuda")
        ws = torch.empty(B.bmnd_match_workspace_size(geom, p.ht), dtype=torch.uint8, device="cuda")
        d_refs = torch.from_numpy(refs).cuda()
        B.bmnd_match(B.STAGE_HT, y, geom, noise, p.ht, d_refs, m, c, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.bmnd_match(B.STAGE_HT, y, geom, noise, p.ht, d_refs, m, c, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"ms": round(dt * 1e3, 3),
                     "mrefs_per_s": round(n_signals * len(refs) / dt / 1e6, 3)}
    B.bmnd_stream_status()
    return {"signals": n_signals, "shape": list(shape), "search": list(w["search"]), **res}


def bench_correlated(B, torch, size: int = 1024, reps: int = 3) -> dict:
    """Stationary correlated Gaussian noise on a 2-D image (Gaussian-filtered
    white noise, sigma 0.1, correlation length 1 px): preparing the tables
    from the spectral density, then the denoise, beside the white-Gaussian
    model on the same input."""
    from paper_2609_34622_amd import synth

    w = WORKLOADS["microscopy-2d-16x1024"]
    shape = (size, size)
    s = synth.correlated_gaussian(shape, seed=8000, sigma=0.1, corr_len=1.0)
    y = torch.from_numpy(np.ascontiguousarray(s.y)).cuda()
    psd = torch.from_numpy(s.psd).cuda()
    geom = B.geometry(shape)
    p = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=w["patch"], step=w["step"], search=w["search"])
    p.ht.group_max, p.wiener.group_max = w["group"]
    tables = B.bmnd_correlated_prepare(psd, geom, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B.bmnd_correlated_prepare(psd, geom, p, tables)
    torch.cuda.synchronize()
    prep = (time.perf_counter() - t0) / reps
    res = {"prepare_ms": round(prep * 1e3, 3), "table_bytes": int(tables.numel())}
    for name, noise in (("correlated", B.correlated(tables)), ("white", B.gaussian(s.sigma))):
        ws = torch.empty(B.bmnd_workspace_size(geom, noise, p), dtype=torch.uint8, device="cuda")
        out = torch.empty_like(y)
        B.bmnd_denoise(y, geom, noise, p, out, None, ws)
        torch.cuda.synchronize()
        B.bmnd_profile_begin()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.bmnd_denoise(y, geom, noise, p, out, None, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        prof = B.bmnd_profile_end()
        res[name] = {"mvox_per_s": round(size * size / dt / 1e6, 3), "ms": round(dt * 1e3, 3),
                     "kernels_ms": {k: round(v[0] / reps, 3) for k, v in prof.items() if v[1]}}
        if name == "correlated":
            o = out.cpu().numpy()
            res["mse_ratio"] = round(float(np.mean((o - s.x) ** 2) / np.mean((s.y - s.x) ** 2)), 4)
        del ws, out
    B.bmnd_stream_status()
    return {"workload": f"image-2d-{size}-correlated", "shape": list(shape),
            "search": list(w["search"]), "group": list(w["group"]), **res}


def _params(B, w):
    p = B.bmnd_params_default(B.PRESET_PLAIN, len(w["shape"]))
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=w["patch"], step=w["step"], search=w["search"])
    p.ht.group_max, p.wiener.group_max = w["group"]
    p.ht.mass_conservation, p.wiener.mass_conservation = map(int, w["mc"])
    return p


def _peak(kernel: str, workload: str):
    """(bound, peak, unit) of a kernel by the instructions it issues: the
    count matchers multiply bytes with v_dot4_u32_u8 (4 multiply-adds per
    lane; the 32-bit integer path runs only where a count exceeds 255, so the
    dot4 rate is the stricter peak); the 1-D filter runs its spatial products
    on the matrix cores (split half precision), every other kernel on the
    FP32 VALU."""
    one_d = workload.startswith("ecg")
    if kernel == "match_ht":
        return "alu", PEAK_DOT4_TOPS, "TOP/s"
    if kernel.startswith("filter") and one_d:
        return "mfma", PEAK_FP32_TFLOPS, "TFLOP/s"
    return "alu", PEAK_FP32_TFLOPS, "TFLOP/s"


def time_workload(B, torch, name: str, steps: int, warmup: int, sample=None, sample_outs=None):
    """Time `steps` complete two-stage denoises of the workload (after
    `warmup` untimed ones) with inputs resident in HBM; returns the JSON
    fields of the line for it."""
    w = WORKLOADS[name]
    y_np, sps = make_input(name, w)
    shape, batch = w["shape"], w["batch"]
    shared = len(set(sps)) == 1 and name.startswith("ecg")
    p = _params(B, w)
    y = torch.from_numpy(y_np).cuda()
    out = torch.empty_like(y)
    pilot = torch.empty_like(y)
    if shared:   # one launch sequence for the whole batch (one noise model)
        calls = [(y, out, pilot, B.geometry(shape, batch), B.poisson(sps[0]))]
    else:        # one call per array, each with its own noise model
        calls = [(y[b], out[b], pilot[b], B.geometry(shape, 1), B.poisson(sps[b]))
                 for b in range(batch)]
    ws = torch.empty(max(B.bmnd_workspace_size(c[3], c[4], p) for c in calls),
                     dtype=torch.uint8, device="cuda")

    def step():
        for yy, oo, pp, gg, nn in calls:
            B.bmnd_denoise(yy, gg, nn, p, oo, pp, ws)

    # ---- block rule of the 2-D / 3-D kernels: autotuned on the first array
    # (every array of the workload has its shape and parameters)
    tuned = None
    if AUTOTUNE and len(shape) in (2, 3):
        yy, oo, pp, gg, nn = calls[0]
        chosen, ms = B.bmnd_autotune(yy, gg, nn, p, oo, ws)
        B.bmnd_stream_status()
        tuned = {"chosen_rule": chosen, "ms_per_rule": [round(m, 3) for m in ms]}

    # ---- algorithmic work per step (group sizes from stage-isolated matching)
    one = B.geometry(shape, 1)
    refs = {B.STAGE_HT: B.bmnd_reference_origins(one, p.ht),
            B.STAGE_WIENER: B.bmnd_reference_origins(one, p.wiener)}
    step()
    B.bmnd_stream_status()
    P = int(np.prod(w["patch"]))
    sj = int(np.sum(w["patch"]))
    F = lambda K: 2 * K * P * sj + 3 * K * P           # one separable transform
    Ks = {B.STAGE_HT: [], B.STAGE_WIENER: []}
    for stage, sp in ((B.STAGE_HT, p.ht), (B.STAGE_WIENER, p.wiener)):
        d_refs = torch.from_numpy(refs[stage]).cuda()
        for yy, oo, pp, gg, nn in calls:
            nb = gg.batch
            m = torch.empty((nb, len(refs[stage]), sp.group_max), dtype=torch.int32, device="cuda")
            c = torch.empty((nb, len(refs[stage])), dtype=torch.int32, device="cuda")
            mws = torch.empty(B.bmnd_match_workspace_size(gg, sp), dtype=torch.uint8, device="cuda")
            B.bmnd_match(stage, yy if stage == B.STAGE_HT else pp, gg, nn, sp, d_refs, m, c, mws)
            B.bmnd_stream_status()
            Ks[stage].append(c.cpu().numpy().astype(np.int64).ravel())
            del m, c, mws
    K_ht, K_wie = np.concatenate(Ks[B.STAGE_HT]), np.concatenate(Ks[B.STAGE_WIENER])
    ncand = {st: candidates_per_ref(shape, w["patch"], w["search"], refs[st]).sum() * batch
             for st in refs}
    sweeps = [2 if m else 1 for m in w["mc"]]   # mass conservation filters twice
    work = {
        "match_ht": 3.0 * P * ncand[B.STAGE_HT],
        "match_wiener": 3.0 * P * ncand[B.STAGE_WIENER],
        "filter_ht": sweeps[0] * float(np.sum(3 * F(K_ht) + 6 * K_ht * P)),
        "filter_wiener": sweeps[1] * float(np.sum(4 * F(K_wie) + 10 * K_wie * P)),
    }
    work_unit = {"match_ht": "int32 VALU ops", "match_wiener": "FP32 flops",
                 "filter_ht": "FP32 flops", "filter_wiener": "FP32 flops"}

    # ---- timed region
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    first = out.clone()
    B.bmnd_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.bmnd_profile_end()
    B.bmnd_stream_status()
    ms_per_step = (t1 - t0) / steps * 1e3
    voxels = batch * int(np.prod(shape))
    value = voxels / (ms_per_step * 1e-3) / 1e6

    # ---- roofline of the dominant kernel: work of a step over its kernel
    # time in a step (the same ratio as per-launch work over launch time)
    per_step = {k: prof[k][0] / steps for k in work}
    dom = max(work, key=lambda k: per_step[k])
    launches = prof[dom][1] / steps
    achieved = work[dom] / (per_step[dom] * 1e-3) / 1e12
    bound, peak, unit = _peak(dom, name)
    roofline = {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                "unit": unit, "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(name, dom),
                "avg_ms": round(per_step[dom] / max(launches, 1), 4),
                "launches_per_step": launches,
                "work_per_launch": work[dom] / max(launches, 1), "work_unit": work_unit[dom]}
    kernels = {k: {"ms_per_step": round(v[0] / steps, 4), "launches": v[1],
                   "frac": (round(work[k] / (v[0] / steps * 1e-3) / 1e12 / _peak(k, name)[1], 4)
                            if k in work and v[0] > 0 else None)}
               for k, v in prof.items() if v[1]}

    # ---- properties of the timed output itself
    checks = {"deterministic": bool(torch.equal(first, out)),
              "finite": bool(torch.isfinite(out).all().item())}
    if w["mc"][1]:
        # mass conservation (Thm. mass conservation): over the samples some
        # group covers (eta > 0), the FP64 numerator over eta sums to the
        # observed total to FP64 round-off, and the float output to its
        # float rounding; samples no group covers stay 0
        fe, oe, unc = [], [], 0
        for yy, oo, pp, gg, nn in calls:
            B.bmnd_denoise(yy, gg, nn, p, oo, pp, ws)
            no, do = B.bmnd_workspace_sums(gg, nn, p)
            nv = yy.numel()
            num = ws[no:no + 8 * nv].view(torch.float64)
            den = ws[do:do + 8 * nv].view(torch.float64)
            cov = den > 0
            yt = yy.reshape(-1).double()[cov].sum()
            fe.append(float(((num[cov] / den[cov]).sum() - yt).abs() / yt))
            oe.append(float((oo.reshape(-1).double()[cov].sum() - yt).abs() / yt))
            unc += int((~cov).sum().item())
        B.bmnd_stream_status()
        checks["mass_fp64_rel_err_max"] = max(fe)
        checks["mass_float_rel_err_max"] = max(oe)
        checks["uncovered_voxels"] = unc

    # ---- the GPU on the oracle's sample (same crops, same parameters),
    # stage by stage: the pilot against the oracle's hard-threshold stage, the
    # output against the oracle's Wiener stage replayed on the GPU's pilot;
    # end to end from y alone is reported beside (the Wiener stage matches
    # on the pilot in float, so candidates tied to round-off may swap)
    val = None
    if sample is not None and sample_outs is not None:
        import oracle as O

        rel = lambda x, r: float(np.abs(x - r).max() / max(np.abs(r).max(), 1e-30))
        pe, we, ee = [], [], []
        for (a, s_p), (ref_pil, ref_out) in zip(sample, sample_outs):
            ad = torch.from_numpy(a).cuda()
            o, pil = B.denoise(ad, B.poisson(s_p), _params(B, w), return_pilot=True)
            B.bmnd_stream_status()
            o = o.cpu().numpy().astype(np.float64)
            pil = pil.cpu().numpy().astype(np.float64)
            _, wie = O.plain_profile(a.shape, w["patch"], w["step"], w["search"], s_p=s_p,
                                     group=w["group"], mc=w["mc"])
            rep = O.run_stage(wie, O.STAGE_WIENER, a, pil)
            pe.append(rel(pil, ref_pil))
            we.append(rel(o, rep))
            ee.append(rel(o, ref_out))
        ok = max(pe) <= REL_ERR_BAR and max(we) <= REL_ERR_BAR
        val = {"pilot_rel_err": max(pe), "wiener_replay_rel_err": max(we),
               "end_to_end_rel_err": max(ee), "per_array_end_to_end": [round(e, 9) for e in ee],
               "bar": REL_ERR_BAR, "pass": ok,
               "sample": "the GPU on the same bounded sample the oracle denoised; A18 max "
                         "|x_gpu - x_orc| / max |x_orc| per array, stage by stage (the Wiener "
                         "stage replayed by the oracle on the GPU's pilot)"}
    del ws, out, pilot, y
    torch.cuda.empty_cache()
    return {"value": round(value, 3), "ms_per_step": round(ms_per_step, 3), "voxels": voxels,
            "config": {"workload": name, "batch": batch, "shape": list(shape),
                       "patch": list(w["patch"]), "step": list(w["step"]),
                       "search": list(w["search"]), "group": list(w["group"]),
                       "profile": "plain", "mass_conservation": list(w["mc"]),
                       "noise": "Poisson, one s_P per array" if not shared else "Poisson, shared s_P",
                       "parallelism": "single GPU", "block_autotune": tuned},
            "roofline": roofline, "kernels": kernels, "output_checks": checks,
            "validation": val}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="phantom-3d-4x256x256x128", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=1,
                    help="time the oracle on a bounded sample and check the GPU against it (0: skip)")
    ap.add_argument("--extra", type=int, default=1,
                    help="also time the other full-size workloads (ECG batch, microscopy stack)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, copy this many MiB device to device once "
                         "(calibrates HBM byte counters under rocprofv3)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="tune the 2-D/3-D block rule on the first array before timing (0: the "
                         "default rule, as the profiling commands run)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests in the serving trace (0: skip the serving comparison)")
    ap.add_argument("--mixed", type=int, default=1,
                    help="also time the batched path and the serving path on mixed 1-D/2-D/3-D "
                         "workloads (0: skip)")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="DB",
                    help="summarize rocprofv3 databases (FETCH_SIZE / WRITE_SIZE runs of a "
                         "--copy-probe-mib bench) into per-launch HBM bytes, print JSON, exit")
    args = ap.parse_args()
    global AUTOTUNE
    AUTOTUNE = bool(args.autotune)
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc, args.copy_probe_mib), indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # the oracle runs first, before anything touches the GPU (its all-core
    # figure forks worker processes)
    sample = outs = cpu = None
    if args.cpu_sample:
        y_np, sps = make_input(args.workload, WORKLOADS[args.workload])
        sample = crops(args.workload, y_np, sps)
        del y_np
        outs, cpu = cpu_baseline(args.workload, sample)
        print(f"oracle sample done: {cpu['sample']}", file=sys.stderr, flush=True)

    import torch

    import paper_2609_34622_amd as B

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    head = time_workload(B, torch, args.workload, args.steps, args.warmup, sample, outs)
    print(f"headline done: {head['value']} Mvox/s", file=sys.stderr, flush=True)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads and writes n floats once
        torch.cuda.synchronize()
        del src, dst

    extra = {}
    if args.extra:
        for name in ("ecg-1d-batch", "microscopy-2d-16x1024"):
            if name == args.workload:
                continue
            r = time_workload(B, torch, name, 3 if name.startswith("micro") else 10, 1)
            extra[name] = {k: r[k] for k in ("value", "ms_per_step", "roofline", "kernels",
                                             "output_checks", "config")}
            extra[name]["unit"] = "Mvox/s"
            print(f"{name} done: {r['value']} Mvox/s", file=sys.stderr, flush=True)

    batched = serving_row = standard = pois = corr = None
    if args.mixed:
        batched = bench_batched(B, torch)
        if args.serving_requests > 0:
            serving_row = bench_serving(B, torch, args.serving_requests)
        standard = bench_standard(B, torch)
        pois = bench_poisson_metrics(B, torch)
        corr = bench_correlated(B, torch)

    line = {
        "metric": METRIC,
        "value": head["value"], "unit": "Mvox/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "arith": "FP32 transforms and shrinkage, FP64 overlap-add sums and mass conservation",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "output_checks": head["output_checks"],
        "validation": head["validation"],
        "cpu_baseline": cpu,
        "extra_workloads": extra,
        "batched": batched,
        "serving": serving_row,
        "standard_profile": standard,
        "poisson_metrics": pois,
        "correlated_gaussian": corr,
    }
    print(json.dumps(line), flush=True)
    if head["validation"] is not None and not head["validation"]["pass"]:
        print("GPU output outside the 1e-4 relative error bar of the oracle", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
