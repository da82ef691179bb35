"""The no-allocation count (cute_count_pairs_noalloc) against cute_count_pairs:
the same counts, bit for bit, on two calls in a row with the second smaller
than the first (the scratch array keeps the first call's contents), for
autocorrelations with tabulated neighbour rows, cross counts and angular
counts without them, counts in host and device memory; the same work
statistics where both calls cut the same home tiles (grids with an explicit
tile size: cute_count_pairs cuts default-size tiles shorter for small counts,
the no-allocation count never does); and the clear rejection of a count whose
temporaries exceed the array."""
import sys

import numpy as np
import pytest

import catalogs
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu


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


def dgrid(cat, geom, r_max, tile_points=64):
    import torch
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for v in (cat.x, cat.y, cat.z)]
    return cute.build_grid(xyz, geom, r_max=r_max, tile_points=tile_points)


STAT_KEYS = ("pair_evals", "pairs_in_range", "retests", "flips", "tiles")


def same(ga, gb, bn, prec, on_device, stats=True):
    import torch
    if on_device:
        o1 = torch.zeros(bn.nbins, dtype=torch.int64, device="cuda")
        o2 = torch.full((bn.nbins,), 7, dtype=torch.int64, device="cuda")
        _, s1 = cute.count_pairs(ga, gb, bn, prec, out=o1, with_stats=True)
        _, s2 = cute.count_pairs_noalloc(ga, gb, bn, prec, out=o2, with_stats=True)
        c1, c2 = o1.cpu().numpy(), o2.cpu().numpy()
    else:
        c1, s1 = cute.count_pairs(ga, gb, bn, prec, with_stats=True)
        c2, s2 = cute.count_pairs_noalloc(ga, gb, bn, prec, with_stats=True)
    np.testing.assert_array_equal(c2.reshape(-1), c1.reshape(-1))
    assert s2["pairs_in_range"] == s1["pairs_in_range"]
    for k in STAT_KEYS if stats else ():
        assert s2[k] == s1[k], (k, s1, s2)
    assert s2["pairs_in_range"] > 0
    return c2


@pytest.mark.parametrize("on_device", [True, False])
def test_noalloc_rmu_auto_two_calls(on_device):
    bn = cute.Binning(cute.BIN_RMU, np.arange(21) * 2.5, np.arange(11) / 10.0, los=cute.LOS_Z)
    big, _ = catalogs.clustered_box_1e6(n_centres=400, per_blob=80, n_rand=10, box=400.0)
    small, _ = catalogs.clustered_box_1e6(n_centres=40, per_blob=50, n_rand=10, box=150.0)
    for name, cat in (("first, 32000 points", big), ("second, 2000 points", small)):
        g = dgrid(cat, cute.GEOM_BOX_OPEN, 50.0)
        for prec in (cute.PREC_FP32_EDGE, cute.PREC_FP64):
            say("noalloc r-mu auto, %s, prec %d, device %d" % (name, prec, on_device))
            same(g, None, bn, prec, on_device)
        g.close()
        # default tile size: cute_count_pairs may cut the tiles shorter
        g = dgrid(cat, cute.GEOM_BOX_OPEN, 50.0, tile_points=0)
        say("noalloc r-mu auto, %s, default tiles, device %d" % (name, on_device))
        same(g, None, bn, cute.PREC_FP32_EDGE, on_device, stats=False)
        g.close()


def test_noalloc_cross_and_angular_two_calls():
    """Cross counts of two open boxes (no tabulated rows: the slots are only
    compacted) and angular counts on the sphere, larger then smaller."""
    bs = cute.Binning(cute.BIN_SIGMAPI, np.arange(16) * 2.0, np.arange(16) * 2.0,
                      los=cute.LOS_MIDPOINT)
    bt = cute.Binning(cute.BIN_THETA, np.deg2rad(np.geomspace(0.01, 3.0, 16)))
    for n_d, n_r in ((20000, 30000), (3000, 2500)):
        say("noalloc sigma-pi cross, %d x %d" % (n_d, n_r))
        d, r = catalogs.lightcone_3e6(n_data=n_d, n_rand=n_r, ra_max_deg=6.0, dec_max_deg=5.0)
        gd = dgrid(d, cute.GEOM_BOX_OPEN, 45.0)
        gr = dgrid(r, cute.GEOM_BOX_OPEN, 45.0)
        same(gd, gr, bs, cute.PREC_FP32_EDGE, True)
        same(gr, gd, bs, cute.PREC_FP64, False)
        say("noalloc theta auto and cross, %d x %d" % (n_d, n_r))
        a, b = catalogs.angular_cap_1e7(n_centres=n_d // 50, per_blob=50, n_rand=n_r,
                                        half_angle_deg=8.0)
        ga = dgrid(a, cute.GEOM_SPHERE, float(bt.edges1[-1]))
        gb = dgrid(b, cute.GEOM_SPHERE, float(bt.edges1[-1]))
        same(ga, None, bt, cute.PREC_FP32_EDGE, True)
        same(ga, gb, bt, cute.PREC_FP32_EDGE, False)
        for g in (gd, gr, ga, gb):
            g.close()


def test_noalloc_rejects_oversize_then_works():
    """A count whose home-tile slots need more than the scratch array is
    rejected with CUTE_E_INVALID_ARG before any work; the next call works."""
    bn = cute.Binning(cute.BIN_MONO, np.arange(11) * 2.0)
    cat = catalogs.uniform_box(1_000_000, 1000.0, seed=77)
    g = dgrid(cat, cute.GEOM_BOX_OPEN, 20.0, tile_points=1)
    say("noalloc oversize: %d one-point tiles" % len(cat))
    with pytest.raises(cute.CuteError) as ei:
        cute.count_pairs_noalloc(g, None, bn, cute.PREC_FP32_EDGE)
    assert ei.value.status == cute.E_INVALID_ARG
    assert "scratch" in str(ei.value)
    g.close()
    small = catalogs.uniform_box(5000, 100.0, seed=78)
    g2 = dgrid(small, cute.GEOM_BOX_OPEN, 20.0)
    say("noalloc after the rejection: 5000 points")
    same(g2, None, bn, cute.PREC_FP32_EDGE, True)
    g2.close()
