"""GPU parity at the limits of one count: the largest histograms that fit
in one workgroup's 160 KB of LDS (one copy, one workgroup per CU), and the
first sizes that do not (a clean CUTE_E_UNSUPPORTED), one-point home tiles,
the limit of 64 points per tile, and catalogs whose steps mostly lie past
the top edge with a few pairs right at it (the step skip), all against the
oracle."""
import sys

import numpy as np
import pytest

import catalogs
import oracle
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu

EXACT = [cute.PREC_FP64, cute.PREC_FP32_EDGE]

# LDS bytes of one count workgroup: the tables (FP64 thresholds and FP32
# bands of both dimensions), four waves' re-test queues, statistics and span
# buffers, and the 64-bit histogram; 160 KB is the per-workgroup maximum.
LDS_MAX = 160 * 1024
PER_WAVE = 12 * 128 + 16 + 12 * 192


def lds_bytes(n1, n2):
    tables = 8 * (n1 + 1) + 8 * (n2 + 1) + 8 * n1 + 8 * max(n2, 1)
    return tables + 4 * PER_WAVE + 8 * n1 * max(n2, 1)


def lds_bytes_h32(n1, n2):
    """The same for the midpoint kinds: 32-bit counters (bytes rounded up to
    8, with 4 more reserved) and 16 bytes for the histogram's budget word."""
    tables = 8 * (n1 + 1) + 8 * (n2 + 1) + 8 * n1 + 8 * max(n2, 1)
    return tables + 4 * PER_WAVE + 16 + 4 + 4 * n1 * max(n2, 1)


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


def test_lds_model_brackets_the_limits():
    assert lds_bytes(6183, 0) <= LDS_MAX < lds_bytes(6184, 0)
    assert lds_bytes(134, 134) <= LDS_MAX < lds_bytes(135, 135)
    assert lds_bytes_h32(188, 188) <= LDS_MAX < lds_bytes_h32(189, 189)


def test_largest_sigmapi_histogram():
    """188 x 188 sigma-pi bins, the most 32-bit counters that fit (one
    workgroup per CU), against the oracle; 189 x 189 is refused."""
    rng = np.random.default_rng(205)
    m = rng.uniform(900.0, 1100.0, (600, 3))
    d = rng.normal(size=(600, 3)) * 8.0
    a = np.concatenate([m, m + d])
    e = np.linspace(0.0, 30.0, 189)
    bn = cute.Binning(cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
    ob = oracle.Binning(oracle.SIGMAPI, e, e, los=oracle.LOS_MID)
    reach = float(np.hypot(30.0, 30.0)) * (1 + 1e-12)
    g = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=reach)
    want = oracle.count_pairs(a, None, ob).reshape(bn.shape)
    assert want.sum() > 0
    for prec in EXACT:
        say("SIGMAPI 188 x 188 bins, prec %d" % prec)
        np.testing.assert_array_equal(cute.count_pairs(g, None, bn, prec), want)
    e2 = np.linspace(0.0, 30.0, 190)
    with pytest.raises(cute.CuteError) as ex:
        cute.count_pairs(g, None, cute.Binning(cute.BIN_SIGMAPI, e2, e2, los=cute.LOS_MIDPOINT))
    assert ex.value.status == cute.E_UNSUPPORTED


@pytest.mark.parametrize("n", [6183])
def test_largest_monopole_histogram(n):
    a = catalogs.mixed_periodic(4000, 200.0, seed=201)
    e = np.linspace(0.0, 60.0, n + 1)
    bn = cute.Binning(cute.BIN_MONO, e)
    want = oracle.count_pairs(a, None, oracle.Binning(oracle.MONO, e))
    g = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=60.0)
    for prec in EXACT:
        say("MONO %d bins, prec %d" % (n, prec))
        np.testing.assert_array_equal(cute.count_pairs(g, None, bn, prec), want)
    with pytest.raises(cute.CuteError) as ex:
        cute.count_pairs(g, None, cute.Binning(cute.BIN_MONO, np.linspace(0.0, 60.0, n + 2)))
    assert ex.value.status == cute.E_UNSUPPORTED


def test_largest_rmu_histogram():
    a = catalogs.mixed_periodic(4000, 200.0, seed=202)
    b = catalogs.uniform_box(3000, 200.0, seed=203)
    e1, e2 = np.linspace(0.0, 50.0, 135), np.linspace(0.0, 1.0, 135)
    bn = cute.Binning(cute.BIN_RMU, e1, e2, los=cute.LOS_Z)
    ob = oracle.Binning(oracle.RMU, e1, e2, los=oracle.LOS_Z)
    ga = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=50.0)
    gb = cute.build_grid(b, cute.GEOM_BOX_OPEN, r_max=50.0)
    want_aa = oracle.count_pairs(a, None, ob).reshape(bn.shape)
    want_ab = oracle.count_pairs(a, b, ob).reshape(bn.shape)
    for prec in EXACT:
        say("RMU 134 x 134 bins, prec %d" % prec)
        np.testing.assert_array_equal(cute.count_pairs(ga, None, bn, prec), want_aa)
        np.testing.assert_array_equal(cute.count_pairs(ga, gb, bn, prec), want_ab)
    big = cute.Binning(cute.BIN_RMU, np.linspace(0.0, 50.0, 136), np.linspace(0.0, 1.0, 136),
                       los=cute.LOS_Z)
    with pytest.raises(cute.CuteError) as ex:
        cute.count_pairs(ga, None, big)
    assert ex.value.status == cute.E_UNSUPPORTED


@pytest.mark.parametrize("tile", [1, 3, 64])
def test_tile_sizes(tile):
    """One-point tiles, a ragged odd size and the 64-point maximum give the
    same counts as the oracle, periodic and open."""
    a = catalogs.mixed_periodic(5000, 300.0, seed=204)
    e = np.linspace(0.0, 40.0, 21)
    for geom, L in ((cute.GEOM_BOX_PERIODIC, 300.0), (cute.GEOM_BOX_OPEN, 0.0)):
        ob = oracle.Binning(oracle.MONO, e, periodic=L > 0, L=L)
        want = oracle.count_pairs(a, None, ob, prune=True)
        g = cute.build_grid(a, geom, box_size=L, r_max=40.0, tile_points=tile)
        for prec in EXACT:
            say("tile %d geom %d prec %d" % (tile, geom, prec))
            np.testing.assert_array_equal(cute.count_pairs(g, None, cute.Binning(cute.BIN_MONO, e),
                                                           prec), want)


def test_tile_slots_after_pool_reuse():
    """Tiles built into per-row slots without a host wait: every slot is
    written, with a tile or as an empty one, also when the memory pool hands
    back blocks that held the tiles of an earlier, larger count. Tile sizes 3
    and 7 put most row boundaries inside a tile, where slots stay empty."""
    big = catalogs.mixed_periodic(60000, 300.0, seed=211)
    small = catalogs.mixed_periodic(4000, 300.0, seed=212)
    e = np.linspace(0.0, 30.0, 16)
    bn = cute.Binning(cute.BIN_MONO, e)
    want = oracle.count_pairs(small, None, oracle.Binning(oracle.MONO, e, periodic=True, L=300.0),
                              prune=True)
    for tile in (3, 7):
        say("slot reuse: tile %d" % tile)
        gb = cute.build_grid(big, cute.GEOM_BOX_PERIODIC, box_size=300.0, r_max=30.0,
                             tile_points=tile)
        assert cute.count_pairs(gb, None, bn, cute.PREC_FP32_EDGE).sum() > 0
        gb.close()
        gs = cute.build_grid(small, cute.GEOM_BOX_PERIODIC, box_size=300.0, r_max=30.0,
                             tile_points=tile)
        for prec in EXACT:
            got, st = cute.count_pairs(gs, None, bn, prec, with_stats=True)
            np.testing.assert_array_equal(got, want)
            assert st["pairs_in_range"] == want.sum()
        gs.close()


def _shell_catalog(rmax, seed, n_blobs=300, per=40, spread=0.5):
    """Blobs whose centres sit at separations close to rmax from other blobs
    (just inside, exactly at, just outside), so that most steps of a count lie
    past the top edge and a few hold single pairs at the edge."""
    rng = np.random.default_rng(seed)
    centres = [np.zeros(3)]
    for k in range(n_blobs - 1):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        f = rng.choice([1.0 - 1e-3, 1.0 - 1e-7, 1.0, 1.0 + 1e-7, 1.0 + 1e-3, 1.5, 2.0])
        centres.append(centres[rng.integers(0, len(centres))] + d * rmax * f)
    c = np.array(centres)
    pts = np.repeat(c, per, axis=0) + rng.normal(scale=spread, size=(len(c) * per, 3))
    pts[::per] = c  # blob centres themselves, so some pairs sit right at the edge
    return pts + 1000.0


@pytest.mark.parametrize("kind", ["mono", "rmu", "sigmapi"])
def test_top_edge_skip_is_exact(kind):
    """Counts where most steps lie past r_max and a few pairs sit at it
    (blob centres at r_max (1 - 1e-7), r_max, r_max (1 + 1e-7)): FP64 and
    FP32_EDGE equal the oracle."""
    rmax = 40.0
    a = _shell_catalog(rmax, 301)
    b = _shell_catalog(rmax, 302)
    if kind == "mono":
        e1, e2, ck, ok, los, olos = np.linspace(0.0, rmax, 9), None, cute.BIN_MONO, oracle.MONO, cute.LOS_Z, oracle.LOS_Z
    elif kind == "rmu":
        e1, e2, ck, ok, los, olos = np.linspace(0.0, rmax, 9), np.linspace(0.0, 1.0, 6), cute.BIN_RMU, oracle.RMU, cute.LOS_Z, oracle.LOS_Z
    else:
        s = rmax / np.sqrt(2.0)
        e1, e2, ck, ok, los, olos = np.linspace(0.0, s, 9), np.linspace(0.0, s, 9), cute.BIN_SIGMAPI, oracle.SIGMAPI, cute.LOS_MIDPOINT, oracle.LOS_MID
    bn = cute.Binning(ck, e1, e2, los=los)
    ob = oracle.Binning(ok, e1, e2, los=olos)
    reach = oracle.rmax(ob)
    ga = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=reach)
    gb = cute.build_grid(b, cute.GEOM_BOX_OPEN, r_max=reach)
    want_aa = oracle.count_pairs(a, None, ob, prune=True).reshape(bn.shape)
    want_ab = oracle.count_pairs(a, b, ob, prune=True).reshape(bn.shape)
    assert want_aa.sum() > 0 and want_ab.sum() > 0
    for prec in EXACT:
        say("top-edge skip, %s, prec %d" % (kind, prec))
        np.testing.assert_array_equal(cute.count_pairs(ga, None, bn, prec), want_aa)
        np.testing.assert_array_equal(cute.count_pairs(ga, gb, bn, prec), want_ab)


def test_allocation_failures_are_reported_and_recovered():
    """The allocation-failure hook (CUTE_TEST_FAIL_ALLOC=n: while set, every
    n-th device allocation of the library reports out-of-memory): grid
    builds, single counts and batches return CUTE_E_OUT_OF_MEMORY at every
    allocation they make, release what they had, and the same calls succeed
    once the hook is cleared, with the oracle's counts."""
    import os
    a = catalogs.uniform_box(3000, 200.0, seed=811)
    e = np.linspace(0.0, 30.0, 7)
    bn = cute.Binning(cute.BIN_MONO, e)
    want = oracle.count_pairs(a, None, oracle.Binning(oracle.MONO, e))
    g = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=30.0)
    seen = set()
    try:
        for n in (1, 2, 3, 5, 8):
            os.environ["CUTE_TEST_FAIL_ALLOC"] = str(n)
            say("allocation failure every %d-th allocation" % n)
            for call in ("grid", "count", "batch"):
                try:
                    if call == "grid":
                        cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=30.0).close()
                    elif call == "count":
                        cute.count_pairs(g, None, bn, cute.PREC_FP32_EDGE)
                    else:
                        cute.count_pairs_batched([cute.BatchItem(g, None, bn)], cute.PREC_FP32_EDGE)
                except cute.CuteError as err:
                    assert err.status == cute.E_OUT_OF_MEMORY, str(err)
                    seen.add(call)
    finally:
        del os.environ["CUTE_TEST_FAIL_ALLOC"]
    assert seen == {"grid", "count", "batch"}
    for prec in EXACT:
        np.testing.assert_array_equal(cute.count_pairs(g, None, bn, prec), want)
    g2 = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=30.0)
    np.testing.assert_array_equal(cute.count_pairs_batched([cute.BatchItem(g2, None, bn)])[0], want)
