"""Serving: continuous batching of denoise requests on one GPU.

Requests of any dimensionality and size arrive over time.  The server
admits a request when an execution slot (one of the server's streams) and enough of the HBM budget are free, uploads its array,
runs the two-stage denoise (``bmnd_denoise``: the noisy input, pilot and
aggregation buffers stay resident on the device across both stages), and
copies the result back.  Requests that arrive while others run are admitted
as slots and memory free up; their kernels overlap on the device.  Each
request's result is exactly the computation of ``bmnd_denoise`` on its own
array, so it does not depend on the mix.

Latency of a request is completion (result back on the host) minus
arrival.  The plain path serves the same trace one request at a time, in
arrival order, on one stream.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import (Params, bmnd_denoise, bmnd_params_default, bmnd_request_bytes,
               bmnd_stream_status, bmnd_workspace_size, geometry, poisson, set_axes, PRESET_PLAIN)
from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the trace start
    y: np.ndarray                  # float32 observation (processing units), array shape
    s_p: float                     # Poisson scale of the observation
    params: Params
    out: Optional[np.ndarray] = None
    admitted: float = float("nan")
    done: float = float("nan")
    nbytes: int = 0                # HBM held while running (request_bytes)
    gap: float = 0.0               # unit-rate arrival gap (set_rate)

    @property
    def voxels(self) -> int:
        return int(self.y.size)


def request_bytes(req: Request, budget: int = 0) -> int:
    """HBM held while the request runs: input and output arrays and the
    denoise workspace (match lists, counts, num/den, pilot), from the
    library; BmndError(E_BUDGET) when it exceeds a nonzero budget."""
    if req.nbytes == 0 or budget:
        geom = geometry(req.y.shape)
        req.nbytes = bmnd_request_bytes(geom, poisson(req.s_p), req.params, budget)
    return req.nbytes


def request_work(req: Request) -> float:
    """Relative cost of a request: reference origins x patch samples x
    (clipped window candidates + a filtering term per group member), the
    scale of both stages' matching and filtering."""
    sp = req.params.ht
    refs = cand = P = 1.0
    for d, L in enumerate(req.y.shape):
        refs *= -(-L // max(sp.step[d], 1))
        cand *= min(sp.search[d], L - sp.patch[d] + 1)
        P *= sp.patch[d]
    return refs * P * (cand + 4.0 * (sp.group_max + req.params.wiener.group_max))


def admits(in_flight: float, work: float, cap: Optional[float], busy: bool) -> bool:
    """Admission rule of the work cap: an idle device takes any request; a
    busy one only while the work in flight stays within the cap."""
    return not busy or cap is None or in_flight + work <= cap


def default_params(ndim: int, mc: bool) -> Params:
    """Per-dimensionality parameters of the mixed workload: 1-D patch 32,
    step 4, search 256, group 16/16; 2-D 8x8, step 3, search 39x39, group
    16/32; 3-D 4x4x4, step 3, search 11^3, group 16/32 (mass conservation
    in 3-D)."""
    p = bmnd_params_default(PRESET_PLAIN, ndim)
    if ndim == 1:
        patch, step, search, group = (32,), (4,), (256,), (16, 16)
    elif ndim == 2:
        patch, step, search, group = (8, 8), (3, 3), (39, 39), (16, 32)
    else:
        patch, step, search, group = (4, 4, 4), (3, 3, 3), (11, 11, 11), (16, 32)
    for sp in (p.ht, p.wiener):
        set_axes(sp, patch=patch, step=step, search=search)
    p.ht.group_max, p.wiener.group_max = group
    p.ht.mass_conservation = p.wiener.mass_conservation = int(mc)
    return p


def make_trace(n: int, rate: float, seed: int, len_1d=(8192, 262144), side_2d=(256, 2048),
               side_3d=(64, 256), mix=(0.4, 0.4, 0.2)) -> List[Request]:
    """Seeded request trace: Poisson arrivals at `rate` requests/s; each
    request a 1-D signal, 2-D image or 3-D volume (probabilities `mix`) with
    log-uniform size in the given ranges and peak log-uniform in [2, 100]
    counts, generated like the batch workloads (ECG signals; disc/rectangle
    or blob/filament images; ellipsoid phantoms)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        kind = rng.choice(3, p=np.asarray(mix) / np.sum(mix))
        peak = float(np.exp(rng.uniform(np.log(2.0), np.log(100.0))))
        s_seed = 5_000_000 + i
        if kind == 0:
            L = int(np.exp(rng.uniform(np.log(len_1d[0]), np.log(len_1d[1]))))
            s = synth.ecg_batch(n_signals=1, length=L, seed=s_seed, peak=peak,
                                baseline=min(5.0, peak / 2))
            y, sp = s.y[0], s.s_p
        elif kind == 1:
            n_side = int(np.exp(rng.uniform(np.log(side_2d[0]), np.log(side_2d[1]))))
            if rng.uniform() < 0.5:
                s = synth.image_2d_small(seed=s_seed, size=n_side, peak=peak)
            else:
                s = synth.microscopy_2d(seed=s_seed, size=n_side)
            y, sp = s.y, s.s_p
        else:
            n_side = int(np.exp(rng.uniform(np.log(side_3d[0]), np.log(side_3d[1]))))
            s = synth.phantom_3d(seed=s_seed, shape=(n_side, n_side, n_side))
            y, sp = s.y, s.s_p
        out.append(Request(i, t, np.ascontiguousarray(y, np.float32), float(sp),
                           default_params(y.ndim, y.ndim == 3)))
    return out


def make_trace_crops(n: int, seed: int, torch, len_1d=(8192, 262144), side_2d=(256, 2048),
                     side_3d=(64, 256), mix=(0.4, 0.4, 0.2), rate: float = float("inf")) -> List[Request]:
    """A large seeded trace built fast: the clean means of a few arrays per
    dimensionality at the largest size (ECG signals; a blob/filament image
    and a disc/rectangle image; an ellipsoid phantom), and per request a
    crop of the drawn size at a seeded offset, rescaled to the request's
    peak (log-uniform in [2, 100] counts) and Poisson-sampled on the device
    with a seeded generator (y = K / peak, s_P = 1 / peak).  Sizes and kinds
    are drawn as in make_trace; arrivals are Poisson at `rate` (inf: all at
    0), with unit-rate gaps kept in `gap` for set_rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b1 = synth.ecg_batch(n_signals=2, length=len_1d[1], seed=seed + 1).x
    b2 = [synth.microscopy_2d(seed=seed + 2, size=side_2d[1]).x,
          synth.image_2d_small(seed=seed + 3, size=side_2d[1]).x]
    b3 = synth.phantom_3d(seed=seed + 4, shape=(side_3d[1],) * 3).x
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    out = []
    for i in range(n):
        gap = float(rng.exponential(1.0))
        kind = rng.choice(3, p=np.asarray(mix) / np.sum(mix))
        peak = float(np.exp(rng.uniform(np.log(2.0), np.log(100.0))))
        if kind == 0:
            L = int(np.exp(rng.uniform(np.log(len_1d[0]), np.log(len_1d[1]))))
            base = b1[int(rng.integers(0, len(b1)))]
            o = int(rng.integers(0, base.shape[0] - L + 1))
            x = base[o:o + L]
        elif kind == 1:
            m = int(np.exp(rng.uniform(np.log(side_2d[0]), np.log(side_2d[1]))))
            base = b2[int(rng.integers(0, 2))]
            o = rng.integers(0, base.shape[0] - m + 1, size=2)
            x = base[o[0]:o[0] + m, o[1]:o[1] + m]
        else:
            m = int(np.exp(rng.uniform(np.log(side_3d[0]), np.log(side_3d[1]))))
            o = rng.integers(0, b3.shape[0] - m + 1, size=3)
            x = b3[o[0]:o[0] + m, o[1]:o[1] + m, o[2]:o[2] + m]
        xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
        lam = xd * (peak / max(float(xd.max().item()), 1e-12))
        y = (torch.poisson(lam, generator=gen) / peak).cpu().numpy()
        r = Request(i, 0.0, np.ascontiguousarray(y, np.float32), 1.0 / peak,
                    default_params(y.ndim, y.ndim == 3))
        r.gap = gap
        out.append(r)
    set_rate(out, rate)
    return out


def set_rate(trace: Sequence[Request], rate: float):
    """Arrival times from the trace's unit-rate gaps at `rate` requests/s
    (inf: every request arrives at 0)."""
    t = 0.0
    for r in trace:
        if np.isfinite(rate):
            t += r.gap / rate
        r.arrival = t if np.isfinite(rate) else 0.0


class _Slot:
    def __init__(self, torch, staging_bytes: int):
        self.stream = torch.cuda.Stream()          # default priority
        self.done = torch.cuda.Event()
        self.req: Optional[Request] = None
        self.bufs = None
        self.host_out = None
        self.bytes = 0
        # pinned staging for the input and the result, allocated once
        n = max(int(staging_bytes) // 4, 1)
        self.pin_in = torch.empty(n, dtype=torch.float32, pin_memory=True)
        self.pin_out = torch.empty(n, dtype=torch.float32, pin_memory=True)


class Server:
    """Continuous batching over `slots` concurrent streams within an HBM
    budget of `budget_bytes`.  A request is admitted only while the work in
    flight (``request_work``) stays within `work_cap`, or when nothing runs:
    small requests still overlap, but two large ones do not stretch each
    other's latency by sharing the device.  The default cap ("auto") is
    half the largest single request seen so far; None admits whatever fits."""

    def __init__(self, budget_bytes: int, slots: int = 4,
                 clock: Callable[[], float] = time.perf_counter,
                 work_cap="auto", staging_bytes: int = 80 << 20):
        import torch

        self.torch = torch
        self.budget = int(budget_bytes)
        self.slots = [_Slot(torch, staging_bytes) for _ in range(slots)]
        # the first work on a new stream sets up its queue: do that now,
        # not inside the first request's latency
        for slot in self.slots:
            with torch.cuda.stream(slot.stream):
                torch.zeros(1, device="cuda")
            slot.stream.synchronize()
        self.clock = clock
        self.work_cap = work_cap
        self.in_use = 0
        self.peak_in_use = 0
        self.work = 0.0
        self.seen_max = 0.0

    def _admit(self, slot: _Slot, req: Request, now: float):
        torch = self.torch
        nbytes = request_bytes(req)
        geom = geometry(req.y.shape)
        noise = poisson(req.s_p)
        n = req.y.size
        staged = n <= slot.pin_in.numel()
        with torch.cuda.stream(slot.stream):
            if staged:
                # the slot's pinned buffers: no host allocation per request
                slot.pin_in[:n].numpy()[:] = req.y.ravel()
                y = slot.pin_in[:n].view(req.y.shape).to("cuda", non_blocking=True)
            else:
                y = torch.from_numpy(req.y).pin_memory().to("cuda", non_blocking=True)
            out = torch.empty_like(y)
            ws = torch.empty(nbytes - 2 * req.y.nbytes, dtype=torch.uint8, device="cuda")
            bmnd_denoise(y, geom, noise, req.params, out, None, ws, stream=slot.stream.cuda_stream)
            if staged:
                host = slot.pin_out[:n].view(req.y.shape)
            else:
                host = torch.empty(out.shape, dtype=torch.float32, pin_memory=True)
            host.copy_(out, non_blocking=True)
            slot.done.record(slot.stream)
        slot.req, slot.bufs, slot.host_out, slot.bytes = req, (y, out, ws), host, nbytes
        req.admitted = now
        self.in_use += nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.work += request_work(req)

    def _retire(self, slot: _Slot, now: float):
        req = slot.req
        req.out = slot.host_out.numpy().copy()
        req.done = now
        self.in_use -= slot.bytes
        self.work = max(self.work - request_work(req), 0.0)
        if all(s.req is None or s is slot for s in self.slots):
            self.work = 0.0
        slot.req, slot.bufs, slot.host_out, slot.bytes = None, None, None, 0

    def run(self, trace: Sequence[Request]) -> dict:
        """Replay `trace` (arrival times relative to the call) and return the
        throughput and latency figures; every request gets `out`, `done`."""
        for r in trace:
            request_bytes(r, self.budget)   # E_BUDGET: never admissible
        pending = deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        t0 = self.clock()
        n_done = 0
        while n_done < len(trace):
            now = self.clock() - t0
            progressed = False
            for slot in self.slots:
                if slot.req is not None and slot.done.query():
                    self._retire(slot, self.clock() - t0)
                    n_done += 1
                    progressed = True
            # admit in arrival order while a slot and the budget allow
            while pending and pending[0].arrival <= now:
                free = [s for s in self.slots if s.req is None]
                if not free or self.in_use + request_bytes(pending[0]) > self.budget:
                    break
                busy = len(free) < len(self.slots)
                w = request_work(pending[0])
                self.seen_max = max(self.seen_max, w)
                cap = 0.5 * self.seen_max if self.work_cap == "auto" else self.work_cap
                if not admits(self.work, w, cap, busy):
                    break
                self._admit(free[0], pending.popleft(), now)
                progressed = True
            if not progressed:
                time.sleep(0.0002)
        bmnd_stream_status(None)
        return summarize(trace)


def serve_fifo(trace: Sequence[Request], clock: Callable[[], float] = time.perf_counter) -> dict:
    """The plain path: one request at a time in arrival order on one stream
    (a request starts when it has arrived and the previous one is done)."""
    import torch

    t0 = clock()
    for req in sorted(trace, key=lambda r: (r.arrival, r.rid)):
        while clock() - t0 < req.arrival:
            time.sleep(0.0002)
        req.admitted = clock() - t0
        geom = geometry(req.y.shape)
        noise = poisson(req.s_p)
        y = torch.from_numpy(req.y).cuda()
        out = torch.empty_like(y)
        ws = torch.empty(bmnd_workspace_size(geom, noise, req.params), dtype=torch.uint8,
                         device="cuda")
        bmnd_denoise(y, geom, noise, req.params, out, None, ws)
        req.out = out.cpu().numpy()
        req.done = clock() - t0
    bmnd_stream_status(None)
    return summarize(trace)


def summarize(trace: Sequence[Request]) -> dict:
    lat = np.array([r.done - r.arrival for r in trace])
    first = min(r.arrival for r in trace)
    last = max(r.done for r in trace)
    vox = sum(r.voxels for r in trace)
    return {
        "requests": len(trace),
        "voxels": int(vox),
        "mvox_per_s": vox / max(last - first, 1e-9) / 1e6,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "makespan_s": float(last - first),
    }
