#!/usr/bin/env python3
"""Throughput of the two-stage BMND hot path on one MI355X.

Workload (default): the 1-D batch -- 256 ECG-like signals of 65536 samples
at 500 Hz, baseline 5 and peak 50 counts, Poisson-sampled; patch 32, step 4,
search window 256, group size 16 in both stages, plain profile, no mass
conservation; all signals in one batched launch sequence.  One step is one
complete two-stage denoise of the whole batch (matching, filtering and
aggregation of both stages), inputs resident in HBM.

Prints one JSON line: metric, value (denoised Mvox/s), roofline of the
dominant kernel (HIP events on the launch stream during the timed region),
and the FP64 oracle timed on a bounded sample on the host cores.
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

PEAK_FP32_TFLOPS = 157.3     # published FP32 vector peak (packed)
PEAK_VALU_TOPS = 78.6        # 32-bit VALU ops/s with a multiply-add counted as 2
PEAK_HBM_GBS = 8000.0

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


def make_input(name: str, w: dict):
    from paper_2609_34622_amd import synth

    if name == "ecg-1d-batch":
        s = synth.ecg_batch(n_signals=w["batch"], length=w["shape"][0], seed=2000)
        return s.y, s.s_p
    if name == "image-2d-128":
        s = synth.image_2d_small(1000)
        return s.y[None], s.s_p
    ys, sps = [], []
    for b in range(w["batch"]):
        if name.startswith("microscopy"):
            s = synth.microscopy_2d(seed=3000 + b, size=w["shape"][0])
        else:
            s = synth.phantom_3d(seed=4000 + b, shape=w["shape"])
        ys.append(s.y)
        sps.append(s.s_p)
    # one noise scale per launch: the batch shares the first array's s_P,
    # the others are rescaled to it (counts preserved exactly)
    y = np.stack([ys[b] / sps[b] * sps[0] for b in range(len(ys))]).astype(np.float32)
    return y, sps[0]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ecg-1d-batch", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=8,
                    help="arrays of the workload the oracle denoises for cpu_baseline (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_34622_amd as B

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = WORKLOADS[args.workload]
    y_np, s_p = make_input(args.workload, w)
    shape, batch = w["shape"], w["batch"]
    y = torch.from_numpy(np.ascontiguousarray(y_np)).cuda()
    geom = B.geometry(shape, batch)
    noise = B.poisson(s_p)
    p = B.bmnd_params_default(B.PRESET_PLAIN, len(shape))
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=w["patch"], step=w["step"], search=w["search"])
    p.ht.group_max, p.wiener.group_max = w["group"]
    p.ht.mass_conservation, p.wiener.mass_conservation = map(int, w["mc"])
    ws = torch.empty(B.bmnd_workspace_size(geom, noise, p), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(y)
    pilot = torch.empty_like(y)

    # ---- algorithmic work per launch (from one untimed stage-isolated pass)
    one = B.geometry(shape, 1)
    refs_ht = B.bmnd_reference_origins(one, p.ht)
    refs_wie = B.bmnd_reference_origins(one, p.wiener)
    B.bmnd_denoise(y, geom, noise, p, out, pilot, ws)
    B.bmnd_stream_status()
    cnt = {}
    for stage, sp, src, refs in ((B.STAGE_HT, p.ht, y, refs_ht), (B.STAGE_WIENER, p.wiener, pilot, refs_wie)):
        m = torch.empty((batch, len(refs), sp.group_max), dtype=torch.int32, device="cuda")
        c = torch.empty((batch, len(refs)), dtype=torch.int32, device="cuda")
        mws = torch.empty(B.bmnd_match_workspace_size(geom, sp), dtype=torch.uint8, device="cuda")
        B.bmnd_match(stage, src, geom, noise, sp, torch.from_numpy(refs).cuda(), m, c, mws)
        B.bmnd_stream_status()
        cnt[stage] = c.cpu().numpy().astype(np.int64)
        del m, c, mws
    P = int(np.prod(w["patch"]))
    sj = int(np.sum(w["patch"]))
    ncand = {B.STAGE_HT: candidates_per_ref(shape, w["patch"], w["search"], refs_ht).sum() * batch,
             B.STAGE_WIENER: candidates_per_ref(shape, w["patch"], w["search"], refs_wie).sum() * batch}
    K_ht, K_wie = cnt[B.STAGE_HT], cnt[B.STAGE_WIENER]
    F = lambda K: 2 * K * P * sj + 3 * K * P           # one separable transform
    work = {
        "match_ht": (3.0 * P * ncand[B.STAGE_HT], "int32 VALU ops"),
        "match_wiener": (3.0 * P * ncand[B.STAGE_WIENER], "FP32 flops"),
        "filter_ht": (float(np.sum(3 * F(K_ht) + 6 * K_ht * P)), "FP32 flops"),
        "filter_wiener": (float(np.sum(4 * F(K_wie) + 10 * K_wie * P)), "FP32 flops"),
    }

    # ---- timed region
    for _ in range(args.warmup):
        B.bmnd_denoise(y, geom, noise, p, out, pilot, ws)
    torch.cuda.synchronize()
    B.bmnd_profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.bmnd_denoise(y, geom, noise, p, out, pilot, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.bmnd_profile_end()
    B.bmnd_stream_status()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    voxels = batch * int(np.prod(shape))
    value = voxels / (ms_per_step * 1e-3) / 1e6

    dom = max((k for k in work), key=lambda k: prof[k][0])
    dom_ms = prof[dom][0] / max(prof[dom][1], 1)
    flops = work[dom][0]
    achieved = flops / (dom_ms * 1e-3) / 1e12
    is_int = work[dom][1].startswith("int32")
    peak = PEAK_VALU_TOPS if is_int else PEAK_FP32_TFLOPS
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TOP/s" if is_int else "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": None, "avg_ms": round(dom_ms, 4),
                "work_per_launch": flops, "work_unit": work[dom][1]}
    kernels = {k: {"ms_per_step": round(v[0] / max(args.steps, 1), 4), "launches": v[1]}
               for k, v in prof.items() if v[1]}

    cpu = None
    if args.cpu_sample > 0:
        import oracle as O

        n = min(args.cpu_sample, batch)
        ht, wie = O.plain_profile(shape, w["patch"], w["step"], w["search"], s_p=s_p,
                                  group=w["group"], mc=w["mc"])
        t0 = time.perf_counter()
        for b in range(n):
            O.denoise(ht, wie, y_np[b])
        dt = time.perf_counter() - t0
        cpu = {"value": round(n * int(np.prod(shape)) / dt / 1e6, 5), "unit": "Mvox/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{n} of {batch} arrays of the same workload, both stages, "
                         f"{dt:.1f} s single-threaded"}

    line = {
        "metric": "denoised Mvox/s (both stages)",
        "value": round(value, 3), "unit": "Mvox/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "batch": batch, "shape": list(shape),
                   "patch": list(w["patch"]), "step": list(w["step"]),
                   "search": list(w["search"]), "group": list(w["group"]),
                   "profile": "plain", "mass_conservation": list(w["mc"]),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
