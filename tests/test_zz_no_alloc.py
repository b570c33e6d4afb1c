"""bmnd_denoise_noalloc (the allocation-free entry point) gives bmnd_denoise's
result, through the C ABI, on two calls in a row on one device (the second
with a smaller input, so it reuses the static scratch the first one filled),
and refuses a denoise larger than its static scratch before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2609_34622_amd as B
from paper_2609_34622_amd import synth

pytestmark = pytest.mark.gpu

REL_OUT = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def _params(shape, patch, step, search, group, mc=False):
    p = B.bmnd_params_default(B.PRESET_PLAIN, len(shape))
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=patch, step=step, search=search)
    p.ht.group_max, p.wiener.group_max = group
    p.ht.mass_conservation = p.wiener.mass_conservation = int(mc)
    return p


def _with_workspace(y, geom, noise, p):
    out = torch.empty_like(y)
    pilot = torch.empty_like(y)
    ws = torch.empty(B.bmnd_workspace_size(geom, noise, p), dtype=torch.uint8, device="cuda")
    B.bmnd_denoise(y, geom, noise, p, out, pilot, ws)
    B.bmnd_stream_status()
    return out.cpu().numpy(), pilot.cpu().numpy()


def _noalloc(y, geom, noise, p, with_pilot):
    out = torch.full_like(y, float("nan"))
    pilot = torch.full_like(y, float("nan")) if with_pilot else None
    stream = int(torch.cuda.current_stream().cuda_stream)
    st = B.lib().bmnd_denoise_noalloc(y.data_ptr(), C.byref(geom), C.byref(noise), C.byref(p),
                                      out.data_ptr(), None if pilot is None else pilot.data_ptr(),
                                      stream)
    assert st == B.OK, B.lib().bmnd_last_error().decode()
    B.bmnd_stream_status()
    return out.cpu().numpy(), None if pilot is None else pilot.cpu().numpy()


def _rel(a, b):
    return float(np.abs(a.astype(np.float64) - b.astype(np.float64)).max()
                 / max(float(np.abs(b).max()), 1e-30))


def _cases():
    big = synth.image_2d_small(1100, size=96)
    small = synth.image_2d_small(1101, size=64)
    rng = np.random.default_rng(7)
    vol_big = (rng.poisson(2.0 + 3.0 * rng.uniform(size=(28, 24, 20))) * 0.2).astype(np.float32)
    vol_small = (rng.poisson(2.0 + 3.0 * rng.uniform(size=(16, 16, 16))) * 0.2).astype(np.float32)
    return [
        ("2-D 96^2 then 64^2",
         (big.y, big.s_p, _params((96, 96), (8, 8), (3, 3), (19, 19), (16, 32))),
         (small.y, small.s_p, _params((64, 64), (8, 8), (3, 3), (19, 19), (16, 32)))),
        ("3-D 28x24x20 then 16^3, mass conservation",
         (vol_big, 0.2, _params((28, 24, 20), (4, 4, 4), (3, 3, 3), (7, 7, 7), (16, 32), mc=True)),
         (vol_small, 0.2, _params((16, 16, 16), (4, 4, 4), (3, 3, 3), (5, 5, 5), (16, 32), mc=True))),
    ]


@pytest.mark.parametrize("case", range(2))
def test_noalloc_equals_denoise_two_calls(case):
    name, first, second = _cases()[case]
    print(f"noalloc case: {name}", flush=True)
    for call, (y_np, s_p, p) in enumerate((first, second)):
        y = torch.from_numpy(np.ascontiguousarray(y_np)).cuda()
        geom = B.geometry(y_np.shape)
        noise = B.poisson(s_p)
        ref_out, ref_pilot = _with_workspace(y, geom, noise, p)
        out, pilot = _noalloc(y, geom, noise, p, with_pilot=(call == 0))
        assert np.all(np.isfinite(out))
        e = _rel(out, ref_out)
        assert e <= REL_OUT, f"call {call}: rel max err {e:.3e} vs bmnd_denoise"
        if pilot is not None:
            assert _rel(pilot, ref_pilot) <= REL_OUT


def test_noalloc_refuses_beyond_its_scratch():
    # a 4096^2 image needs far more than the static scratch: refused on the
    # host, before any copy or launch
    shape = (4096, 4096)
    geom = B.geometry(shape)
    p = _params(shape, (8, 8), (3, 3), (19, 19), (16, 32))
    y = torch.zeros(16, dtype=torch.float32, device="cuda")  # never read
    st = B.lib().bmnd_denoise_noalloc(y.data_ptr(), C.byref(geom), C.byref(B.poisson(0.1)),
                                      C.byref(p), y.data_ptr(), None,
                                      int(torch.cuda.current_stream().cuda_stream))
    assert st == B.E_WORKSPACE
    assert "scratch" in B.lib().bmnd_last_error().decode()
