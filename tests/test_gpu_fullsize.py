"""Parity at the full sizes of the light-cone (sigma-pi) and angular workloads.

The oracle cannot count these catalogs whole, so the checks are
  * sampled outputs: the cross counts of 64 seeded home points against the
    whole other catalog (the rows of DR and DD that those points own), which
    the oracle computes one home point set at a time, bit-exact;
  * properties that hold at any size: the FP32_EDGE counts equal the FP64
    counts of the same full-size autocorrelation.
Inputs are the full-size seeded catalogs of both workloads."""
import sys

import numpy as np
import pytest

import catalogs
import oracle
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu

EXACT = [cute.PREC_FP64, cute.PREC_FP32_EDGE]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    cute.load()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dgrid(cat, geom, r_max):
    import torch
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for v in (cat.x, cat.y, cat.z)]
    return cute.build_grid(xyz, geom, r_max=r_max)


def sample(cat, n, seed):
    idx = np.sort(np.random.Generator(np.random.PCG64(seed)).choice(len(cat), n, replace=False))
    return cat.subset(idx)


def test_sigmapi_lightcone_full_size():
    """3e6 data and 6e6 randoms in the light cone; sigma and pi edges 2k Mpc/h
    (k <= 75), midpoint line of sight."""
    say("generating the light-cone catalogs")
    d, r = catalogs.config3()
    e = np.arange(76) * 2.0
    bn = cute.Binning(cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
    ob = oracle.Binning(oracle.SIGMAPI, e, e, los=oracle.LOS_MID)
    rmax = oracle.rmax(ob)
    gd = dgrid(d, cute.GEOM_BOX_OPEN, rmax)
    gr = dgrid(r, cute.GEOM_BOX_OPEN, rmax)
    s = sample(d, 64, seed=31)
    gs = cute.build_grid(s, cute.GEOM_BOX_OPEN, r_max=rmax)
    for other, go, name in ((r, gr, "S x R"), (d, gd, "S x D")):
        want = oracle.count_pairs(s, other, ob, prune=True)
        assert want.sum() > 0
        for prec in EXACT:
            say("sigma-pi full size: %s prec %d" % (name, prec))
            got = cute.count_pairs(gs, go, bn, prec)
            np.testing.assert_array_equal(got, want, err_msg="%s prec %d" % (name, prec))
    say("sigma-pi full size: DD FP32_EDGE vs FP64")
    c32, st = cute.count_pairs(gd, None, bn, cute.PREC_FP32_EDGE, with_stats=True)
    c64 = cute.count_pairs(gd, None, bn, cute.PREC_FP64)
    np.testing.assert_array_equal(c32, c64)
    say("sigma-pi full size: DD %d pairs in range, %d evaluations, %.1f ms"
        % (st["pairs_in_range"], st["pair_evals"], st["ms_count"]))
    assert st["pairs_in_range"] > 0


def test_theta_cap_full_size():
    """1e7 clustered data and 2e7 randoms in a 5000 sq-deg cap; 30 log bins of
    theta in [0.001, 10] degrees."""
    say("generating the angular catalogs")
    d, r = catalogs.config4()
    e = np.deg2rad(0.001 * 10.0 ** (np.arange(31) * 4.0 / 30.0))
    bn = cute.Binning(cute.BIN_THETA, e)
    ob = oracle.Binning(oracle.THETA, e)
    gd = dgrid(d, cute.GEOM_SPHERE, e[-1])
    gr = dgrid(r, cute.GEOM_SPHERE, e[-1])
    s = sample(d, 64, seed=41)
    gs = cute.build_grid(s, cute.GEOM_SPHERE, r_max=e[-1])
    for other, go, name in ((r, gr, "S x R"), (d, gd, "S x D")):
        want = oracle.count_pairs(s, other, ob, prune=True)
        assert want.sum() > 0
        for prec in EXACT:
            say("theta full size: %s prec %d" % (name, prec))
            got = cute.count_pairs(gs, go, bn, prec)
            np.testing.assert_array_equal(got, want, err_msg="%s prec %d" % (name, prec))
    # the full autocorrelation of a tenth of the data: FP32_EDGE == FP64
    sub = sample(d, len(d) // 10, seed=42)
    gsub = dgrid(sub, cute.GEOM_SPHERE, e[-1])
    say("theta full size: DD of %d points, FP32_EDGE vs FP64" % len(sub))
    c32, st = cute.count_pairs(gsub, None, bn, cute.PREC_FP32_EDGE, with_stats=True)
    c64 = cute.count_pairs(gsub, None, bn, cute.PREC_FP64)
    np.testing.assert_array_equal(c32, c64)
    say("theta: %d pairs in range, %d evaluations, %.1f ms"
        % (st["pairs_in_range"], st["pair_evals"], st["ms_count"]))
