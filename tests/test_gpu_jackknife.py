"""GPU parity of the jackknife by region decomposition (cute_count_jackknife).

Each jackknife row must equal the oracle's autocorrelation of the catalog
without that region (bit-exact for FP64 and FP32_EDGE), the masked batched
count of the same catalog, and the total the plain autocorrelation. Inputs:
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
