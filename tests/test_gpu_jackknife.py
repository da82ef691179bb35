"""GPU parity of the jackknife by region decomposition (cute_count_jackknife
and, for cross-correlations, cute_count_jackknife_cross).

Each jackknife row must equal the oracle's count of the catalog(s) without
that region (bit-exact for FP64 and FP32_EDGE), the masked batched count of
the same catalog(s), and the total the plain count. Inputs:
the batched mock workload's shapes (periodic box, half uniform half
clustered, 10 x 10 column regions) and clustered data in an open box with
slab regions, at sizes the oracle finishes in seconds."""
import sys

import numpy as np
import pytest

import catalogs
import oracle
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu

EXACT = [cute.PREC_FP64, cute.PREC_FP32_EDGE]
L = 1000.0


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


def bins_periodic():
    return [(cute.Binning(cute.BIN_MONO, np.arange(31) * 5.0),
             oracle.Binning(oracle.MONO, np.arange(31) * 5.0, periodic=True, L=L)),
            (cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, np.arange(51) / 50.0),
             oracle.Binning(oracle.RMU, np.arange(41) * 5.0, np.arange(51) / 50.0,
                            los=oracle.LOS_Z, periodic=True, L=L))]


def test_jackknife_periodic_columns_match_oracle():
    _, base, region = catalogs.batched_mocks_256(n_mocks=1, n_lo=100, n_hi=200, jk_base=5000, box=L)
    g = cute.build_grid(base, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0)
    for bn, ob in bins_periodic():
        want_total = oracle.count_pairs(base, None, ob).reshape(-1)
        checked = [0, 1, 9, 44, 90, 99]
        want = {k: oracle.count_pairs(base.subset(np.nonzero(region != k)[0]), None, ob).reshape(-1)
                for k in checked}
        for prec in EXACT:
            say("jackknife periodic, %d bins, prec %d" % (bn.nbins, prec))
            total, jack = cute.count_jackknife(g, region, 100, bn, prec)
            np.testing.assert_array_equal(total.reshape(-1), want_total)
            for k in checked:
                np.testing.assert_array_equal(jack[k].reshape(-1), want[k], err_msg="region %d" % k)
            # every row against the masked batch (one item per region)
            items = [cute.BatchItem(g, None, bn, mask_a=(region == k).astype(np.uint8))
                     for k in range(100)]
            got = cute.count_pairs_batched(items, prec)
            for k in range(100):
                np.testing.assert_array_equal(jack[k], got[k], err_msg="region %d" % k)


def test_jackknife_open_box_slabs_and_edge_cases():
    d, _ = catalogs.clustered_box_1e6(n_centres=120, per_blob=30, n_rand=10, box=300.0)
    # 7 slabs in x, one of them empty
    xs = (d.x - d.x.min()) / (d.x.max() - d.x.min() + 1e-9)
    region = np.minimum((xs * 6).astype(np.int32), 5)
    region[region == 3] = 6          # region 3 stays empty
    K = 7
    bn = cute.Binning(cute.BIN_RMU, np.linspace(0, 40, 9), np.linspace(0, 1, 11))
    ob = oracle.Binning(oracle.RMU, np.linspace(0, 40, 9), np.linspace(0, 1, 11), los=oracle.LOS_Z)
    g = cute.build_grid(d, cute.GEOM_BOX_OPEN, r_max=40.0)
    for prec in EXACT:
        total, jack = cute.count_jackknife(g, region, K, bn, prec)
        np.testing.assert_array_equal(total, oracle.count_pairs(d, None, ob))
        for k in range(K):
            keep = np.nonzero(region != k)[0]
            np.testing.assert_array_equal(jack[k], oracle.count_pairs(d.subset(keep), None, ob),
                                          err_msg="region %d prec %d" % (k, prec))
        np.testing.assert_array_equal(jack[3], total)  # the empty region removes nothing
    # one region holding everything: its jackknife catalog is empty
    total, jack = cute.count_jackknife(g, np.zeros(len(d), np.int32), 1, bn)
    assert jack.sum() == 0 and total.sum() > 0
    # device labels, and a label out of range
    import torch
    total2, jack2 = cute.count_jackknife(g, torch.from_numpy(region).cuda(), K, bn)
    np.testing.assert_array_equal(total2, total)
    bad = region.copy()
    bad[5] = K
    with pytest.raises(cute.CuteError):
        cute.count_jackknife(g, bad, K, bn)


def test_jackknife_cross_periodic_matches_oracle_and_masks():
    """Cross jackknife (cute_count_jackknife_cross) of two periodic catalogs
    with 10 x 10 column regions: every row equals the masked batched cross
    count, sampled rows and the total equal the oracle."""
    _, base, region = catalogs.batched_mocks_256(n_mocks=1, n_lo=100, n_hi=200, jk_base=4000, box=L)
    other = catalogs.mixed_periodic(3000, L, seed=7101)
    ix = np.minimum((other.x * (10.0 / L)).astype(np.int64), 9)
    iy = np.minimum((other.y * (10.0 / L)).astype(np.int64), 9)
    reg_b = (iy * 10 + ix).astype(np.int32)
    ga = cute.build_grid(base, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0)
    gb = cute.build_grid(other, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=200.0)
    for bn, ob in bins_periodic():
        want_total = oracle.count_pairs(base, other, ob).reshape(bn.shape)
        checked = [0, 7, 44, 99]
        want = {k: oracle.count_pairs(base.subset(np.nonzero(region != k)[0]),
                                      other.subset(np.nonzero(reg_b != k)[0]), ob).reshape(bn.shape)
                for k in checked}
        for prec in EXACT:
            say("cross jackknife periodic, %d bins, prec %d" % (bn.nbins, prec))
            total, jack = cute.count_jackknife_cross(ga, region, gb, reg_b, 100, bn, prec)
            np.testing.assert_array_equal(total, want_total)
            for k in checked:
                np.testing.assert_array_equal(jack[k], want[k], err_msg="region %d" % k)
            items = [cute.BatchItem(ga, gb, bn, mask_a=(region == k).astype(np.uint8),
                                    mask_b=(reg_b == k).astype(np.uint8)) for k in range(100)]
            got = cute.count_pairs_batched(items, prec)
            for k in range(100):
                np.testing.assert_array_equal(jack[k], got[k], err_msg="region %d" % k)


def test_jackknife_cross_open_boxes_of_different_extent():
    """Clustered data against uniform randoms in open boxes of different
    bounding boxes (so the neighbour rows are derived per tile), 6 slab
    regions with one empty in the randoms, against the oracle; device labels;
    the same grid twice is rejected."""
    import torch
    d, r = catalogs.clustered_box_1e6(n_centres=100, per_blob=30, n_rand=4000, box=300.0)
    reg_d = np.minimum(((d.x - d.x.min()) / (np.ptp(d.x) + 1e-9) * 6).astype(np.int32), 5)
    reg_r = np.minimum(((r.x - r.x.min()) / (np.ptp(r.x) + 1e-9) * 6).astype(np.int32), 5)
    reg_r[reg_r == 2] = 4             # region 2 of the randoms is empty
    K = 6
    e1, e2 = np.linspace(0, 40, 9), np.linspace(0, 1, 11)
    bn = cute.Binning(cute.BIN_RMU, e1, e2)
    ob = oracle.Binning(oracle.RMU, e1, e2, los=oracle.LOS_Z)
    gd = cute.build_grid(d, cute.GEOM_BOX_OPEN, r_max=40.0)
    gr = cute.build_grid(r, cute.GEOM_BOX_OPEN, r_max=40.0)
    for prec in EXACT:
        say("cross jackknife open boxes, prec %d" % prec)
        total, jack = cute.count_jackknife_cross(gd, reg_d, gr, reg_r, K, bn, prec)
        np.testing.assert_array_equal(total, oracle.count_pairs(d, r, ob))
        for k in range(K):
            want = oracle.count_pairs(d.subset(np.nonzero(reg_d != k)[0]),
                                      r.subset(np.nonzero(reg_r != k)[0]), ob)
            np.testing.assert_array_equal(jack[k], want, err_msg="region %d prec %d" % (k, prec))
    t2, j2 = cute.count_jackknife_cross(gd, torch.from_numpy(reg_d).cuda(), gr,
                                        torch.from_numpy(reg_r).cuda(), K, bn)
    np.testing.assert_array_equal(j2, jack)
    with pytest.raises(cute.CuteError) as ex:
        cute.count_jackknife_cross(gd, reg_d, gd, reg_d, K, bn)
    assert ex.value.status == cute.E_INVALID_ARG


def test_jackknife_lattice_ties_match_oracle():
    """A dyadic lattice in a periodic box of side 12 (pairs exactly on the r
    and mu edges) split into 8 regions by octant: every leave-one-out count
    equals the oracle's count of the lattice without that region."""
    Ll = 12.0
    e1, e2 = np.arange(0, 9) * 0.5, np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    g = np.random.Generator(np.random.PCG64(29))
    pts = g.integers(0, 24, size=(2500, 3)).astype(np.float64) * 0.5
    region = ((pts[:, 0] >= 6.0).astype(np.int32) + 2 * (pts[:, 1] >= 6.0) + 4 * (pts[:, 2] >= 6.0)).astype(np.int32)
    grid = cute.build_grid(pts, cute.GEOM_BOX_PERIODIC, box_size=Ll, r_max=4.0)
    for bn, ob in ((cute.Binning(cute.BIN_MONO, e1), oracle.Binning(oracle.MONO, e1, periodic=True, L=Ll)),
                   (cute.Binning(cute.BIN_RMU, e1, e2, los=cute.LOS_Z),
                    oracle.Binning(oracle.RMU, e1, e2, los=oracle.LOS_Z, periodic=True, L=Ll))):
        want_total = oracle.count_pairs(pts, None, ob).reshape(-1)
        for prec in EXACT:
            say("jackknife lattice, %d bins, prec %d" % (bn.nbins, prec))
            total, jack = cute.count_jackknife(grid, region, 8, bn, prec)
            np.testing.assert_array_equal(total.reshape(-1), want_total)
            for k in range(8):
                want = oracle.count_pairs(pts[region != k], None, ob).reshape(-1)
                np.testing.assert_array_equal(jack[k].reshape(-1), want, err_msg="region %d" % k)
