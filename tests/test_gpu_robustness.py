"""Non-finite inputs on the GPU path: the library stays memory-safe, the
matching kernels keep every listed member valid, count-domain matching
reports the bad samples, and outputs far from them are unaffected."""
import numpy as np
import pytest
import torch

import paper_2609_34622_amd as B
from paper_2609_34622_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def _params(shape, patch, step, search, group):
    p = B.bmnd_params_default(B.PRESET_PLAIN, len(shape))
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=patch, step=step, search=search)
    p.ht.group_max, p.wiener.group_max = group
    return p


def _lists_valid(m, c, shape, patch, gmax):
    ell = [shape[d] - patch[d] for d in range(len(shape))]
    for g in range(c.size):
        K = int(c.flat[g])
        assert K >= 1 and K <= gmax and (K & (K - 1)) == 0, K
        row = m.reshape(-1, gmax)[g]
        assert np.all(row[K:] == -1)
        for lin in row[:K]:
            assert lin >= 0
            co = np.unravel_index(int(lin), shape)
            assert all(co[d] <= ell[d] for d in range(len(shape)))


CASES = [((4096,), (32,), (4,), (256,), (16, 16)),
         ((40, 36), (8, 8), (3, 3), (15, 15), (16, 32))]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_nonfinite_pilot_lists_valid(case):
    shape, patch, step, search, group = case
    print(f"non-finite Wiener matching {shape}", flush=True)
    rng = np.random.default_rng(7)
    src = rng.uniform(0.0, 1.0, size=shape).astype(np.float32)
    bad = rng.choice(src.size, size=max(4, src.size // 200), replace=False)
    src.flat[bad[::2]] = np.nan
    src.flat[bad[1::2]] = np.inf
    p = _params(shape, patch, step, search, group)
    geom = B.geometry(shape)
    refs = B.bmnd_reference_origins(geom, p.wiener)
    n = len(refs)
    m = torch.empty((1, n, p.wiener.group_max), dtype=torch.int32, device="cuda")
    c = torch.empty((1, n), dtype=torch.int32, device="cuda")
    ws = torch.empty(B.bmnd_match_workspace_size(geom, p.wiener), dtype=torch.uint8, device="cuda")
    B.bmnd_match(B.STAGE_WIENER, torch.from_numpy(src).cuda(), geom, B.poisson(0.02), p.wiener,
                 torch.from_numpy(refs).cuda(), m, c, ws)
    B.bmnd_stream_status()
    _lists_valid(m.cpu().numpy(), c.cpu().numpy(), shape, patch, p.wiener.group_max)


def _denoise(y, geom, noise, p):
    yd = torch.from_numpy(y).cuda()
    ws = torch.empty(B.bmnd_workspace_size(geom, noise, p), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(yd)
    B.bmnd_denoise(yd, geom, noise, p, out, None, ws)
    return out


def test_nonfinite_observation_1d():
    print("non-finite observation 1-D 4096", flush=True)
    s = synth.ecg_batch(n_signals=1, length=4096, seed=2003)
    shape, patch, step, search = (4096,), (32,), (4,), (256,)
    p = _params(shape, patch, step, search, (16, 16))
    geom = B.geometry(shape)
    clean = _denoise(s.y, geom, B.poisson(s.s_p), p)
    B.bmnd_stream_status()
    clean = clean.cpu().numpy()
    y = s.y.copy()
    y[0, 2000] = np.nan
    # count-domain HT matching reports the sample ...
    out = _denoise(y, geom, B.poisson(s.s_p), p)
    with pytest.raises(B.BmndError):
        B.bmnd_stream_status()
    B.bmnd_stream_status()  # flag cleared
    # ... and the plain-SSD (Gaussian) path runs through; the damage stays local
    sig = float(np.sqrt(s.s_p * max(float(s.y.mean()), 1e-6)))
    clean_g = _denoise(s.y, geom, B.gaussian(sig), p).cpu().numpy()
    out_g = _denoise(y, geom, B.gaussian(sig), p)
    B.bmnd_stream_status()
    out_g = out_g.cpu().numpy()
    far = np.ones(4096, bool)
    far[2000 - 900:2000 + 900] = False
    assert np.all(np.isfinite(out_g[0, far]))
    # float atomics accumulate in any order, and a last-bit change of the
    # pilot may flip a Wiener near-tie: nearly all far samples agree to 1e-5,
    # all of them to 1e-3
    scale = np.abs(clean_g).max()
    d = np.abs(out_g[0, far] - clean_g[0, far])
    assert np.mean(d <= 1e-5 * scale) >= 0.99
    assert d.max() <= 1e-3 * scale
    del out, clean
