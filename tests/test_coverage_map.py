"""Coverage map C(x) of the reference schedules and its coefficient of
variation (section Experiments, Shift Schedule Analysis), on the CPU.

The oracle counts, for every scheduled origin, the samples of its patch; it
is pinned here by hand-worked cases, the tiling case (CV = 0), the total
count invariant and an independent numpy evaluation (box sums by cumulative
sums over an origin indicator).  The library's separable computation is
then compared with the oracle map by map, and with the committed table of
the workload shapes."""
import os

import numpy as np
import pytest

import oracle as O
import paper_2609_34622_amd as B

HERE = os.path.dirname(os.path.abspath(__file__))


def _stage(shape, patch, step, sched="generated", rho=2.0, ks=2):
    return O.Stage(shape=shape, patch=patch, step=step, search=(1,) * len(shape),
                   schedule=sched, shift_density=rho, passes=ks)


def _numpy_coverage(shape, patch, origins):
    """C(x) = #{r : x in r + B} as box sums of the origin indicator, by
    cumulative sums along each axis (independent of the oracle's loop)."""
    ind = np.zeros(shape, np.int64)
    ind.ravel()[origins] = 1
    c = ind
    for d, j in enumerate(patch):
        cs = np.cumsum(c, axis=d)
        shifted = np.zeros_like(cs)
        sl_dst = [slice(None)] * len(shape)
        sl_src = [slice(None)] * len(shape)
        sl_dst[d] = slice(j, None)
        sl_src[d] = slice(0, shape[d] - j)
        shifted[tuple(sl_dst)] = cs[tuple(sl_src)]
        c = cs - shifted
    return c


def test_oracle_coverage_hand_1d():
    # L 10, patch 4, step 3, unshifted: origins 0, 3, 6 (ell = 6 is the last slot)
    st = _stage((10,), (4,), (3,), sched="off")
    assert O.schedule(st).tolist() == [0, 3, 6]
    cov, mean, sd, cv = O.coverage(st)
    assert cov.tolist() == [1, 1, 1, 2, 1, 1, 2, 1, 1, 1]
    # mean 12/10; deviations: eight of -0.2, two of +0.8 -> variance 0.16
    assert mean == pytest.approx(1.2, abs=1e-15)
    assert sd == pytest.approx(0.4, abs=1e-15)
    assert cv == pytest.approx(1.0 / 3.0, abs=1e-15)


def test_oracle_coverage_hand_2d_clipped_last_slot():
    # 7 x 5, patch 3 x 2, step 3 x 2, unshifted: rows 0, 3, 4 (ell 4 pinned),
    # columns 0, 2, 3 (ell 3 pinned)
    st = _stage((7, 5), (3, 2), (3, 2), sched="off")
    rows, cols = [0, 3, 4], [0, 2, 3]
    assert sorted(O.schedule(st).tolist()) == sorted(r * 5 + c for r in rows for c in cols)
    row_cov = [1, 1, 1, 1, 2, 2, 1]          # patches at rows 0, 3, 4 of height 3
    col_cov = [1, 1, 1, 2, 1]                # patches at columns 0, 2, 3 of width 2
    cov, mean, sd, cv = O.coverage(st)
    assert cov.tolist() == [[r * c for c in col_cov] for r in row_cov]
    vals = np.outer(row_cov, col_cov).astype(float)
    assert mean == pytest.approx(vals.sum() / 35, abs=1e-15)
    assert sd == pytest.approx(np.sqrt(((vals - vals.mean()) ** 2).mean()), abs=1e-15)


@pytest.mark.parametrize("shape,patch", [((12,), (4,)), ((12, 8), (4, 4)), ((9, 6, 4), (3, 3, 2))])
def test_oracle_coverage_tiling_is_uniform(shape, patch):
    # step = patch and patch | shape: the patches tile the array, C = 1 everywhere
    st = _stage(shape, patch, patch, sched="off")
    cov, mean, sd, cv = O.coverage(st)
    assert (cov == 1).all()
    assert mean == 1.0 and sd == 0.0 and cv == 0.0


@pytest.mark.parametrize("sched,rho,ks", [("off", 0.0, 1), ("generated", 2.0, 2),
                                          ("generated", 1.0, 1), ("balanced", 2.0, 2),
                                          ("balanced", 4.0, 2), ("sparse", 2.0, 2)])
@pytest.mark.parametrize("shape,patch,step", [((64, 48), (8, 8), (3, 3)),
                                              ((37, 41), (8, 8), (3, 3)),
                                              ((20, 18, 16), (4, 4, 4), (3, 3, 3)),
                                              ((30, 1, 26), (4, 1, 4), (3, 1, 3)),
                                              ((2000,), (32,), (4,)),
                                              ((6, 7, 8, 9), (2, 3, 4, 2), (2, 2, 3, 1))])
def test_oracle_coverage_equals_numpy(sched, rho, ks, shape, patch, step):
    st = _stage(shape, patch, step, sched, rho, ks)
    origins = O.schedule(st)
    cov, mean, sd, cv = O.coverage(st)
    ref = _numpy_coverage(shape, patch, origins)
    assert np.array_equal(cov.astype(np.int64), ref)
    # every origin contributes one patch: sum C = |R| |B|
    assert int(cov.sum()) == len(origins) * int(np.prod(patch))
    assert mean == pytest.approx(ref.mean(), rel=1e-14)
    assert sd == pytest.approx(ref.std(), rel=1e-12, abs=1e-14)
    assert cv == pytest.approx(ref.std() / ref.mean(), rel=1e-12, abs=1e-14)


def _lib_coverage(shape, patch, step, sched, rho, ks):
    sp = B.bmnd_params_default(0, min(len(shape), 3)).ht
    B.set_axes(sp, patch=patch, step=step, search=(1,) * len(shape))
    sp.schedule = B.SCHED[sched]
    sp.shift_density = rho
    sp.passes = ks
    return B.bmnd_reference_coverage(B.geometry(shape), sp)


@pytest.mark.parametrize("sched,rho,ks", [("off", 0.0, 1), ("generated", 2.0, 2),
                                          ("balanced", 2.0, 2), ("balanced", 1.0, 2),
                                          ("sparse", 2.0, 2)])
@pytest.mark.parametrize("shape,patch,step", [((128, 128), (8, 8), (3, 3)),
                                              ((37, 41), (8, 8), (3, 3)),
                                              ((40, 36, 28), (4, 4, 4), (3, 3, 3)),
                                              ((40, 1, 50), (8, 1, 8), (3, 1, 3)),
                                              ((65536,), (32,), (4,)),
                                              ((6, 7, 8, 9), (2, 3, 4, 2), (2, 2, 3, 1))])
def test_library_coverage_equals_oracle(sched, rho, ks, shape, patch, step):
    cov, mean, sd, cv = _lib_coverage(shape, patch, step, sched, rho, ks)
    ocov, omean, osd, ocv = O.coverage(_stage(shape, patch, step, sched, rho, ks))
    assert np.array_equal(cov, ocov)
    tol = max(1e-12, float(np.prod(shape)) * 2.0 ** -52)   # FP64 sums over |Omega|
    assert mean == pytest.approx(omean, rel=tol)
    assert sd == pytest.approx(osd, rel=tol, abs=1e-14)
    assert cv == pytest.approx(ocv, rel=tol, abs=1e-14)


def _table():
    rows = []
    with open(os.path.join(HERE, "golden", "coverage_e01.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, sched, rho, ks, n, mean, sd, cv = line.split()
            rows.append((name, sched, float(rho), int(ks), int(n), float(mean), float(sd),
                         float(cv)))
    return rows


SHAPES = {"image-128": ((128, 128), (8, 8), (3, 3)), "image-256": ((256, 256), (8, 8), (3, 3)),
          "image-512": ((512, 512), (8, 8), (3, 3)),
          "image-481x321": ((481, 321), (8, 8), (3, 3)),
          "image-768x512": ((768, 512), (8, 8), (3, 3)),
          "microscopy-1024": ((1024, 1024), (8, 8), (3, 3)),
          "phantom-256x256x128": ((256, 256, 128), (4, 4, 4), (3, 3, 3)),
          "ecg-65536": ((65536,), (32,), (4,))}


def test_library_reproduces_schedule_table():
    """Reference counts and coverage CV of every schedule on the workload
    shapes (the geometric half of the schedule analysis) from the library,
    against the table the oracle wrote."""
    rows = _table()
    assert len(rows) == len(SHAPES) * 12
    for name, sched, rho, ks, n, mean, sd, cv in rows:
        shape, patch, step = SHAPES[name]
        _, lmean, lsd, lcv = _lib_coverage(shape, patch, step, sched, rho, ks)
        sp = B.bmnd_params_default(0, len(shape)).ht
        B.set_axes(sp, patch=patch, step=step, search=(1,) * len(shape))
        sp.schedule, sp.shift_density, sp.passes = B.SCHED[sched], rho, ks
        assert len(B.bmnd_reference_origins(B.geometry(shape), sp)) == n, (name, sched, rho, ks)
        # the oracle sums |Omega| squared deviations in FP64 one by one:
        # relative round-off up to about |Omega| 2^-53 (the library sums by
        # histogram)
        tol = max(1e-12, float(np.prod(shape)) * 2.0 ** -52)
        assert lmean == pytest.approx(mean, rel=tol)
        assert lcv == pytest.approx(cv, rel=tol, abs=1e-14), (name, sched, rho, ks)


def test_schedule_table_observations():
    """Properties of the table that the schedule analysis reports: the
    standard generated (2, 2) schedule and the unshifted single pass on the
    workload shapes, and balanced (2, 2) spreading its references more
    evenly than generated (2, 2) on the 2-D images."""
    rows = {(r[0], r[1], r[2], r[3]): r for r in _table()}
    # counts quoted for the workloads: generated (2, 2) and unshifted
    assert rows[("image-128", "generated", 2.0, 2)][4] == 3216
    assert rows[("microscopy-1024", "generated", 2.0, 2)][4] == 229976
    assert rows[("phantom-256x256x128", "generated", 2.0, 2)][4] == 308890
    assert rows[("ecg-65536", "generated", 2.0, 2)][4] == 16377
    assert rows[("image-128", "off", 0.0, 1)][4] == 1681
    # sparse = generated without singleton axes: identical on these shapes
    for name in SHAPES:
        assert rows[(name, "sparse", 2.0, 2)][4:] == rows[(name, "generated", 2.0, 2)][4:]
    for name in ("image-256", "image-512", "image-481x321", "image-768x512", "microscopy-1024"):
        assert rows[(name, "balanced", 2.0, 2)][7] < rows[(name, "generated", 2.0, 2)][7]
        assert rows[(name, "balanced", 2.0, 2)][4] < rows[(name, "generated", 2.0, 2)][4]
