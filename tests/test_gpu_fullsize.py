"""Parity at the full sizes of the light-cone (sigma-pi), angular and batched
workloads.

The oracle cannot count these catalogs whole, so the checks are
  * sampled outputs: the cross counts of 64 seeded home points against the
    whole other catalog (the rows of DR and DD that those points own), which
    the oracle computes one home point set at a time, bit-exact;
  * properties that hold at any size: the FP32_EDGE counts equal the FP64
    counts of the same full-size counts (sigma-pi DD, DR and RR; the angular
    DD).
Inputs are the full-size seeded catalogs of the three workloads."""
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


def dgrid(cat, geom, r_max, L=0.0):
    import torch
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for v in (cat.x, cat.y, cat.z)]
    return cute.build_grid(xyz, geom, box_size=L, r_max=r_max)


def sample(cat, n, seed):
    idx = np.sort(np.random.Generator(np.random.PCG64(seed)).choice(len(cat), n, replace=False))
    return cat.subset(idx)


def test_sigmapi_lightcone_full_size():
    """3e6 data and 6e6 randoms in the light cone; sigma and pi edges 2k Mpc/h
    (k <= 75), midpoint line of sight."""
    say("generating the light-cone catalogs")
    d, r = catalogs.lightcone_3e6()
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
    for name, ga, gb in (("DD", gd, None), ("DR", gd, gr), ("RR", gr, None)):
        say("sigma-pi full size: %s FP32_EDGE vs FP64" % name)
        c32, st = cute.count_pairs(ga, gb, bn, cute.PREC_FP32_EDGE, with_stats=True)
        c64 = cute.count_pairs(ga, gb, bn, cute.PREC_FP64)
        np.testing.assert_array_equal(c32, c64, err_msg=name)
        say("sigma-pi full size: %s %d pairs in range, %d evaluations, %.1f ms"
            % (name, st["pairs_in_range"], st["pair_evals"], st["ms_count"]))
        assert st["pairs_in_range"] > 0


def test_theta_cap_full_size():
    """1e7 clustered data and 2e7 randoms in a 5000 sq-deg cap; 30 log bins of
    theta in [0.001, 10] degrees."""
    say("generating the angular catalogs")
    d, r = catalogs.angular_cap_1e7()
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
    # the full 1e7-point autocorrelation: FP32_EDGE == FP64
    say("theta full size: DD of %d points, FP32_EDGE vs FP64" % len(d))
    c32, st = cute.count_pairs(gd, None, bn, cute.PREC_FP32_EDGE, with_stats=True)
    c64 = cute.count_pairs(gd, None, bn, cute.PREC_FP64)
    np.testing.assert_array_equal(c32, c64)
    say("theta: %d pairs in range, %d evaluations, %.1f ms"
        % (st["pairs_in_range"], st["pair_evals"], st["ms_count"]))


def test_batched_mocks_and_jackknife_full_size():
    """The batched workload at full size: 256 periodic mocks (2e4 .. 5e5
    points) with the monopole binning and jackknife catalogs of the 1e6-point
    base with the r-mu binning, in one batch per precision. FP32_EDGE equals
    FP64 item by item; sampled mocks equal their single counts; the smallest
    mock equals the oracle; each jackknife catalog satisfies
    DD(base) = DD(rest) + DD(region) + DR(rest, region)."""
    import torch
    L = 1000.0
    say("generating the batched workload")
    mocks, base, region = catalogs.batched_mocks_256()
    mono = cute.Binning(cute.BIN_MONO, np.arange(31) * 5.0)
    rmu = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, np.arange(51) / 50.0, los=cute.LOS_Z)
    gm = [dgrid(m, cute.GEOM_BOX_PERIODIC, 200.0, L) for m in mocks]
    gb = dgrid(base, cute.GEOM_BOX_PERIODIC, 200.0, L)
    gb2 = dgrid(base, cute.GEOM_BOX_PERIODIC, 200.0, L)
    items = [cute.BatchItem(g, None, mono) for g in gm]
    regs = [0, 57, 99]
    for r in regs:
        m = torch.from_numpy((region == r).astype(np.uint8)).cuda()
        items += [cute.BatchItem(gb, None, rmu, mask_a=m),
                  cute.BatchItem(gb, None, rmu, mask_a=1 - m),
                  cute.BatchItem(gb, gb2, rmu, mask_a=m, mask_b=1 - m)]
    res = {}
    for prec in EXACT:
        say("full-size batch, prec %d, %d items" % (prec, len(items)))
        res[prec], st = cute.count_pairs_batched(items, prec, with_stats=True)
        say("  %.1f ms, %d pair evaluations" % (st["ms_count"], st["pair_evals"]))
    for k in range(len(items)):
        np.testing.assert_array_equal(res[cute.PREC_FP32_EDGE][k], res[cute.PREC_FP64][k],
                                      err_msg="item %d" % k)
    got = res[cute.PREC_FP32_EDGE]
    sizes = np.array([len(m) for m in mocks])
    for k in list(np.argsort(sizes)[::32]) + [int(np.argmax(sizes))]:
        np.testing.assert_array_equal(got[k], cute.count_pairs(gm[k], None, mono,
                                                               cute.PREC_FP32_EDGE))
    k0 = int(np.argmin(sizes))
    ob = oracle.Binning(oracle.MONO, np.arange(31) * 5.0, periodic=True, L=L)
    np.testing.assert_array_equal(got[k0], oracle.count_pairs(mocks[k0], None, ob, prune=True))
    dd_base = cute.count_pairs(gb, None, rmu, cute.PREC_FP32_EDGE)
    for q, r in enumerate(regs):
        rest, reg, cross = got[len(gm) + 3 * q: len(gm) + 3 * q + 3]
        np.testing.assert_array_equal(rest + reg + cross, dd_base, err_msg="region %d" % r)


def test_rmu_dr_rr_full_size_and_estimators():
    """The r-mu workload at its full size beyond DD: 1e6 clustered data and
    2e6 uniform randoms. The DR and RR rows of 64 seeded sample points equal
    the oracle's; the full DR and RR in FP32_EDGE equal FP64; Landy-Szalay
    xi(r, mu) and its multipoles from the full counts agree with the oracle's
    exact-rational estimators to 1e-12."""
    import json
    import os

    from oracle import estimators as est
    d, r = catalogs.clustered_box_1e6()
    e1, e2 = np.arange(41) * 5.0, np.arange(51) / 50.0
    bn = cute.Binning(cute.BIN_RMU, e1, e2, los=cute.LOS_Z)
    ob = oracle.Binning(oracle.RMU, e1, e2, los=oracle.LOS_Z)
    gd = dgrid(d, cute.GEOM_BOX_OPEN, 200.0)
    gr = dgrid(r, cute.GEOM_BOX_OPEN, 200.0)
    for cat, name in ((d, "D"), (r, "R")):
        s = sample(cat, 64, seed=51 if name == "D" else 52)
        gs = cute.build_grid(s, cute.GEOM_BOX_OPEN, r_max=200.0)
        want = oracle.count_pairs(s, r, ob, prune=True).reshape(bn.shape)
        for prec in EXACT:
            say("r-mu full size: %s-sample x R, prec %d" % (name, prec))
            np.testing.assert_array_equal(cute.count_pairs(gs, gr, bn, prec), want)
    say("r-mu full size: DR and RR, FP32_EDGE vs FP64")
    dr = cute.count_pairs(gd, gr, bn, cute.PREC_FP32_EDGE)
    np.testing.assert_array_equal(dr, cute.count_pairs(gd, gr, bn, cute.PREC_FP64))
    rr = cute.count_pairs(gr, None, bn, cute.PREC_FP32_EDGE)
    np.testing.assert_array_equal(rr, cute.count_pairs(gr, None, bn, cute.PREC_FP64))
    golden = os.path.join(os.path.dirname(__file__), "golden", "clustered_1e6_dd_rmu.json")
    with open(golden) as f:
        dd = np.array(json.load(f)["counts"], dtype=np.uint64).reshape(bn.shape)
    nd, nr = len(d), len(r)
    say("r-mu full size: Landy-Szalay and multipoles")
    xi = cute.xi_estimate(cute.EST_LS, dd, dr, rr, nd, nr, bn)
    want = est.landy_szalay(dd, dr, rr, nd, nr)
    ok = ~np.isnan(want)
    assert ok.all() and np.array_equal(np.isnan(xi), np.isnan(want))
    rel = np.abs(xi[ok] - want[ok]) / np.maximum(np.abs(want[ok]), 1e-300)
    assert rel.max() <= 1e-12, rel.max()
    ells = (0, 2, 4)
    got_m = cute.xi_multipoles(xi, bn, ells)
    want_m = est.multipoles(want, e2, list(ells))
    for a, ell in enumerate(ells):
        scale = np.abs(want) @ est.multipole_weights_abs(e2, ell)
        assert np.all(np.abs(got_m[a] - want_m[a]) <= 1e-12 * scale + 1e-300)
