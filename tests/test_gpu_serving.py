"""Serving by continuous batching: every request's result is the same alone
and in the mix (1e-4 relative, the output tolerance), admission respects
the HBM budget, and the plain one-at-a-time path agrees."""
import numpy as np
import pytest
import torch

import paper_2609_34622_amd as B
from paper_2609_34622_amd import serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def _alone(req):
    geom = B.geometry(req.y.shape)
    noise = B.poisson(req.s_p)
    y = torch.from_numpy(req.y).cuda()
    out = torch.empty_like(y)
    ws = torch.empty(B.bmnd_workspace_size(geom, noise, req.params), dtype=torch.uint8,
                     device="cuda")
    B.bmnd_denoise(y, geom, noise, req.params, out, None, ws)
    B.bmnd_stream_status()
    return out.cpu().numpy()


def _trace(n=14, rate=400.0, seed=77):
    return serving.make_trace(n, rate, seed, len_1d=(2048, 8192), side_2d=(48, 96),
                              side_3d=(16, 24))


def _rel(a, b):
    return float(np.abs(a.astype(np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


def test_serving_same_alone_and_in_mix():
    print("serving mix of 14 requests", flush=True)
    trace = _trace()
    assert {r.y.ndim for r in trace} == {1, 2, 3}
    alone = [_alone(r) for r in trace]
    budget = sum(serving.request_bytes(r) for r in trace)
    srv = serving.Server(budget_bytes=budget, slots=4)
    stats = srv.run(trace)
    assert stats["requests"] == len(trace)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    for r, a in zip(trace, alone):
        assert r.out is not None and r.out.shape == r.y.shape
        assert r.done >= r.arrival
        assert _rel(r.out, a) < 1e-4, r.rid
    assert srv.in_use == 0


def test_serving_budget_limits_admission():
    print("serving under a tight HBM budget", flush=True)
    trace = _trace(n=8, seed=78)
    biggest = max(serving.request_bytes(r) for r in trace)
    srv = serving.Server(budget_bytes=biggest + biggest // 2, slots=4)
    srv.run(trace)
    assert srv.peak_in_use <= biggest + biggest // 2
    for r in trace:
        assert _rel(r.out, _alone(r)) < 1e-4, r.rid
    with pytest.raises(B.BmndError) as e:
        serving.Server(budget_bytes=biggest // 2).run(trace[:1] + [max(trace, key=serving.request_bytes)])
    assert e.value.status == B.E_BUDGET


def test_fifo_path_agrees():
    print("plain one-at-a-time path", flush=True)
    trace = _trace(n=6, seed=79)
    stats = serving.serve_fifo(trace)
    assert stats["requests"] == 6
    for r in trace:
        assert _rel(r.out, _alone(r)) < 1e-4, r.rid
