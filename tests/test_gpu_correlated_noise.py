"""GPU parity under stationary correlated Gaussian noise (section
Observation Models; Prop. Gaussian SSD noise bias; Lemma covariance
propagation) against the FP64 oracle, which builds the group covariance
from numpy's inverse FFT of the spectral density and propagates it with the
full transform.

Replay protocol as in the other parity tests.  Tolerances:
  * HT lists: identical, except where two FP64 scores (or a score and the
    threshold) agree to 1e-12 of the term magnitude: the autocovariance
    comes from different code on the two sides (the library's partial DFT,
    numpy's FFT), so the bias may differ in the last bits;
  * filtered patches: 2e-5 of the group's largest |p|;
  * weights 1e-5, and for the Wiener stage also the bound that FP32 pilot
    transforms put on them: correlated noise gives some coefficients a
    variance far below c(0), and their gain G = Gamma^2 / (Gamma^2 + s_v v)
    then responds to pilot coefficients Gamma near the FP32 round-off of the
    group, |dGamma| <= 1e-6 ||gamma_g||; with dG = 2 G (1 - G) dGamma / Gamma
    the classic surrogate R = sum G^2 moves by at most
    sum 4 G^2 (1 - G) |dGamma / Gamma|;
  * denoised arrays: 1e-4 of the largest |value|.
Shapes cover every kernel: the N-D matcher and the cube filter (8x8, 4x4x4,
32-sample 1-D patches), the generic matcher and filter (6x5 patches).

The noise spectra keep their smallest value above about 1e-6 of the largest
(correlation lengths up to 1.2 samples): where a coefficient's propagated
variance falls to FP64 round-off of c(0), both sides hold rounding noise
and the Wiener gain of such a coefficient is not reproducible."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_2609_34622_amd as B
from paper_2609_34622_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_OUT = 1e-4
REL_PATCH = 2e-5

CASES = {
    # name: shape, patch, step, search, corr_len, group (HT, Wiener)
    "2d-8x8": ((30, 28), (8, 8), (3, 3), (11, 11), (1.0, 1.2), (16, 16)),
    "2d-6x5": ((30, 28), (6, 5), (3, 2), (9, 11), (1.2, 0.7), (8, 16)),
    "3d-4": ((13, 12, 11), (4, 4, 4), (3, 3, 3), (5, 5, 5), (0.8, 1.0, 1.2), (8, 16)),
    "1d-32": ((1000,), (32,), (4,), (48,), (1.2,), (16, 16)),
}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def rel_err(a, ref):
    return float(np.abs(np.asarray(a, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-30))


def setup(name, seed=8100, sigma=0.1):
    shape, patch, step, search, cl, group = CASES[name]
    s = synth.correlated_gaussian(shape, seed=seed, sigma=sigma, corr_len=cl)
    p = B.bmnd_params_default(B.PRESET_PLAIN, len(shape))
    for sp in (p.ht, p.wiener):
        B.set_axes(sp, patch=patch, step=step, search=search)
    p.ht.group_max, p.wiener.group_max = group
    geom = B.geometry(shape)
    tables = B.bmnd_correlated_prepare(dev(s.psd, torch.float64), geom, p)
    noise = B.correlated(tables)
    ht, wie = O.plain_profile(shape, patch, step, search, group=group, noise="correlated",
                              psd=s.psd)
    return s, p, geom, noise, ht, wie


def gpu_match(stage, src, geom, noise, sp, refs):
    n = len(refs)
    m = torch.empty((geom.batch, n, sp.group_max), dtype=torch.int32, device="cuda")
    c = torch.empty((geom.batch, n), dtype=torch.int32, device="cuda")
    ws = torch.empty(B.bmnd_match_workspace_size(geom, sp), dtype=torch.uint8, device="cuda")
    B.bmnd_match(stage, src, geom, noise, sp, dev(refs, torch.int64), m, c, ws)
    B.bmnd_stream_status()
    return m.cpu().numpy(), c.cpu().numpy()


def gpu_filter(stage, y, pilot, geom, noise, sp, match, count):
    b, n, g = match.shape
    P = int(np.prod([sp.patch[d] for d in range(geom.ndim)]))
    pt = torch.empty((b, n, g, P), dtype=torch.float32, device="cuda")
    wt = torch.empty((b, n, g), dtype=torch.float32, device="cuda")
    B.bmnd_filter(stage, y, pilot, geom, noise, sp, n, dev(match, torch.int32),
                  dev(count, torch.int32), pt, wt)
    B.bmnd_stream_status()
    return pt.cpu().numpy(), wt.cpu().numpy()


def gpu_denoise(y, geom, noise, params):
    ws = torch.empty(B.bmnd_workspace_size(geom, noise, params), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(y)
    pilot = torch.empty_like(y)
    B.bmnd_denoise(y, geom, noise, params, out, pilot, ws)
    B.bmnd_stream_status()
    return out.cpu().numpy(), pilot.cpu().numpy()


def _scores(y, shape, patch, acov, gamma, r, lins):
    """FP64 corrected SSD of candidates (numpy) for the tie analysis."""
    P = int(np.prod(patch))
    rc = np.unravel_index(int(r), shape)
    pr = y[tuple(slice(rc[d], rc[d] + patch[d]) for d in range(len(shape)))].astype(np.float64)
    out = []
    for lin in lins:
        cc = np.unravel_index(int(lin), shape)
        q = y[tuple(slice(cc[d], cc[d] + patch[d]) for d in range(len(shape)))].astype(np.float64)
        dl = tuple((cc[d] - rc[d]) % shape[d] for d in range(len(shape)))
        out.append(((q - pr) ** 2).sum() - gamma * 2.0 * P * (acov[(0,) * len(shape)] - acov[dl]))
    return np.array(out)


def check_lists(y, shape, patch, acov, gamma, tau, mg, cg, mo, co):
    bad = []
    for g in range(len(co)):
        if cg[g] == co[g] and np.array_equal(mg[g, :cg[g]], mo[g, :co[g]]):
            continue
        r = mo[g, 0]
        lins = sorted((set(mg[g, 1:cg[g]]) | set(mo[g, 1:co[g]])) - {-1})
        sc = dict(zip(lins, _scores(y, shape, patch, acov, gamma, r, lins)))
        mag = max(1.0, max(abs(v) for v in sc.values()), abs(tau))
        tie = lambda a, b: abs(a - b) <= 1e-12 * mag
        if cg[g] != co[g]:
            if not any(tie(v, tau) for v in sc.values()):
                bad.append(g)
            continue
        K = co[g]
        kth = sc[mo[g, K - 1]]
        for lin in set(mg[g, 1:K]) ^ set(mo[g, 1:K]):
            if not tie(sc[lin], kth):
                bad.append(g)
        sg = [sc[lin] for lin in mg[g, 1:K]]
        if any(sg[i + 1] < sg[i] and not tie(sg[i], sg[i + 1]) for i in range(len(sg) - 1)):
            bad.append(g)
    return bad


@pytest.mark.parametrize("name", list(CASES))
def test_correlated_ht_lists(name):
    _say(f"correlated HT lists {name}")
    s, p, geom, noise, ht, wie = setup(name)
    shape, patch = CASES[name][0], CASES[name][1]
    refs = B.bmnd_reference_origins(geom, p.ht)
    mg, cg = gpu_match(B.STAGE_HT, dev(s.y), geom, noise, p.ht, refs)
    mo, co, _, _ = O.match(ht, O.STAGE_HT, s.y, s.y, refs)
    tau = 3000.0 * ht.P / 255.0 ** 2
    bad = check_lists(s.y, shape, patch, O.autocovariance(s.psd), 3.0, tau, mg[0], cg[0], mo, co)
    assert not bad, (len(bad), bad[:5])
    assert (cg[0] > 2).any()


def wiener_weight_rtol(st, pilot, org):
    """Relative bound on the classic Wiener weight from FP32 pilot
    transforms (module docstring), from the oracle's FP64 coefficients."""
    gam, var, _, _ = O.group_coeffs(st, O.STAGE_WIENER, pilot, pilot, org)
    gam, var = gam.ravel(), np.maximum(var.ravel(), 0.0)
    sh = gam ** 2
    den = sh + st.s_v * var
    G = np.where(den > 0, sh / np.where(den > 0, den, 1.0), 0.0)
    R = float(np.sum(G ** 2))
    dgam = 1e-6 * float(np.sqrt(np.sum(gam ** 2)))
    with np.errstate(divide="ignore", invalid="ignore"):
        dR = np.where(np.abs(gam) > 0, 4 * G ** 2 * (1 - G) * dgam / np.abs(gam), 0.0)
    return float(np.sum(dR)) / R if R > 0 else 0.0


@pytest.mark.parametrize("stage", ["ht", "wiener"])
@pytest.mark.parametrize("name", list(CASES))
def test_correlated_filter(name, stage):
    """Patches and weights on the GPU's own lists against the oracle's."""
    _say(f"correlated filter {name} {stage}")
    s, p, geom, noise, ht, wie = setup(name)
    wien = stage == "wiener"
    sp = p.wiener if wien else p.ht
    st_id = B.STAGE_WIENER if wien else B.STAGE_HT
    refs = B.bmnd_reference_origins(geom, sp)
    pilot = s.x if wien else None
    src = dev(pilot) if wien else dev(s.y)
    mg, cg = gpu_match(st_id, src, geom, noise, sp, refs)
    pg, wg = gpu_filter(st_id, dev(s.y), None if pilot is None else dev(pilot), geom, noise, sp,
                        mg, cg)
    po, wo = O.filter(wie if wien else ht, O.STAGE_WIENER if wien else O.STAGE_HT, s.y, pilot,
                      mg[0], cg[0])
    for g in range(len(refs)):
        K = cg[0, g]
        scale = max(np.abs(po[g, :K]).max(), 1e-30)
        assert np.abs(pg[0, g, :K] - po[g, :K]).max() <= REL_PATCH * scale, g
        rtol = 1e-5
        if wien:
            rtol += wiener_weight_rtol(wie, pilot, mg[0, g, :K])
        assert np.allclose(wg[0, g, :K], wo[g, :K], rtol=rtol, atol=0), (g, rtol)


@pytest.mark.parametrize("name", list(CASES))
def test_correlated_denoise(name):
    _say(f"correlated denoise {name}")
    s, p, geom, noise, ht, wie = setup(name)
    out, pilot = gpu_denoise(dev(s.y), geom, noise, p)
    pil_o = O.run_stage(ht, O.STAGE_HT, s.y)
    assert rel_err(pilot, pil_o) < REL_OUT
    out_o = O.run_stage(wie, O.STAGE_WIENER, s.y, pilot.astype(np.float64))
    assert rel_err(out, out_o) < REL_OUT


def test_correlated_batch_and_mismatch():
    """Two arrays of one shape share the tables; tables prepared for other
    stage parameters are refused."""
    _say("correlated batch")
    name = "2d-8x8"
    s, p, geom, noise, ht, wie = setup(name)
    s2 = synth.correlated_gaussian(CASES[name][0], seed=8200, sigma=0.1, corr_len=CASES[name][4])
    y2 = np.stack([s.y, s2.y])
    g2 = B.geometry(CASES[name][0], batch=2)
    out, pilot = gpu_denoise(dev(y2), g2, noise, p)
    out1, _ = gpu_denoise(dev(s.y), geom, noise, p)
    assert np.allclose(out[0], out1, rtol=1e-6, atol=1e-7)
    other = B.bmnd_params_default(B.PRESET_PLAIN, 2)
    for sp in (other.ht, other.wiener):
        B.set_axes(sp, patch=CASES[name][1], step=CASES[name][2], search=(13, 13))
    with pytest.raises(B.BmndError):
        gpu_denoise(dev(s.y), geom, noise, other)
