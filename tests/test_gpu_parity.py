"""GPU parity: the HIP pair counter (through the C ABI) against the CPU FP64
oracle, element by element on the same seeded inputs.

Counts are integers, so the bar is bit-exact equality for FP64 and FP32_EDGE.
FP32_ONLY is not exact; its miscounts are bounded by the flips that the
FP32_EDGE path reports (each misclassified pair moves one count)."""
import json
import math
import os
import sys

import numpy as np
import pytest

import catalogs
import oracle
import paper_1210_1833_amd as cute
from oracle import estimators as est

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
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


def ocat(c):
    return c


def obin(kind, e1, e2=None, los=cute.LOS_Z, periodic=False, L=0.0):
    ok = {cute.BIN_MONO: oracle.MONO, cute.BIN_RMU: oracle.RMU, cute.BIN_SIGMAPI: oracle.SIGMAPI,
          cute.BIN_THETA: oracle.THETA}[kind]
    ol = oracle.LOS_Z if los == cute.LOS_Z else oracle.LOS_MID
    return oracle.Binning(ok, e1, e2, los=ol, periodic=periodic, L=L)


def gpu_counts(a, b, binning, prec, geom, L=0.0, r_max=0.0, cell=0.0, stats=False):
    ga = cute.build_grid(a, geom, box_size=L, r_max=r_max, cell_size=cell)
    gb = None if b is None else cute.build_grid(b, geom, box_size=L, r_max=r_max, cell_size=cell)
    return cute.count_pairs(ga, gb, binning, prec, with_stats=stats)


def check_case(name, a, b, kind, e1, e2=None, los=cute.LOS_Z, geom=cute.GEOM_BOX_OPEN, L=0.0,
               cell=0.0, precs=EXACT, prune=False):
    bn = cute.Binning(kind, e1, e2, los=los)
    rmax = oracle.rmax(obin(kind, e1, e2, los))
    want = oracle.count_pairs(a, b, obin(kind, e1, e2, los, geom == cute.GEOM_BOX_PERIODIC, L),
                              prune=prune).reshape(bn.shape)
    assert want.sum() > 0 or len(a) < 2
    for prec in precs:
        say("case %s prec %d n_a %d n_b %s" % (name, prec, len(a), None if b is None else len(b)))
        got, st = gpu_counts(a, b, bn, prec, geom, L=L,
                             r_max=(bn.edges1[-1] if kind == cute.BIN_THETA else rmax),
                             cell=cell, stats=True)
        assert got.dtype == np.uint64
        np.testing.assert_array_equal(got, want, err_msg="%s prec %d" % (name, prec))
        assert st["pairs_in_range"] == int(want.sum())
    return want


# ---------------------------------------------------------------------------
def test_mono_periodic_auto_and_cross():
    a = catalogs.uniform_box(6000, 300.0, seed=101)
    b = catalogs.mixed_periodic(5000, 300.0, seed=102)
    e = np.linspace(0.0, 45.0, 16)
    check_case("mono-periodic-auto", a, None, cute.BIN_MONO, e, geom=cute.GEOM_BOX_PERIODIC, L=300.0)
    check_case("mono-periodic-cross", a, b, cute.BIN_MONO, e, geom=cute.GEOM_BOX_PERIODIC, L=300.0)


def test_mono_periodic_2e4_full_size():
    """20 000 uniform points in a periodic box of side 1000 at full size,
    against the oracle's brute force."""
    with open(os.path.join(GOLDEN, "periodic_2e4_dd_mono.json")) as f:
        g = json.load(f)
    c = catalogs.periodic_uniform_2e4()
    assert catalogs.sha256_of(c) == g["sha256"]
    bn = cute.Binning(cute.BIN_MONO, np.array(g["r_edges"]))
    for prec in EXACT:
        say("case periodic-2e4 prec", prec)
        got = gpu_counts(c, None, bn, prec, cute.GEOM_BOX_PERIODIC, L=1000.0, r_max=150.0)
        np.testing.assert_array_equal(got, np.array(g["counts"], dtype=np.uint64))


def test_rmu_dd_full_size_benchmark_workload():
    """The benchmark workload at its full size (1e6 clustered points, r-mu
    40 x 50 bins) in the benchmark's launch configuration, against the
    oracle's counts stored by tests/golden/make_golden.py."""
    import torch
    with open(os.path.join(GOLDEN, "clustered_1e6_dd_rmu.json")) as f:
        g = json.load(f)
    d, _ = catalogs.clustered_box_1e6()
    assert catalogs.sha256_of(d) == g["sha256"], "generator output changed"
    want = np.array(g["counts"], dtype=np.uint64)
    dev = torch.device("cuda:0")
    xyz = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (d.x, d.y, d.z)]
    bn = cute.Binning(cute.BIN_RMU, np.array(g["r_edges"]), np.array(g["mu_edges"]), los=cute.LOS_Z)
    out = torch.zeros(bn.nbins, dtype=torch.int64, device=dev)
    for prec in EXACT:
        say("case c2-full prec", prec)
        grid = cute.build_grid(xyz, cute.GEOM_BOX_OPEN, r_max=200.0)
        _, st = cute.count_pairs(grid, None, bn, prec, out=out, with_stats=True)
        np.testing.assert_array_equal(out.cpu().numpy().astype(np.uint64), want)
        assert st["pairs_in_range"] == int(want.sum())
    # the FP32-only path misclassifies only a few pairs per million
    cute.count_pairs(grid, None, bn, cute.PREC_FP32_ONLY, out=out)
    l1 = int(np.abs(out.cpu().numpy() - want.astype(np.int64)).sum())
    assert l1 < 1e-4 * int(want.sum())


@pytest.mark.parametrize("cell", [0.0, 7.0, 33.0])
def test_mono_open_log_bins(cell):
    d, r = catalogs.clustered_box_1e6(n_centres=120, per_blob=40, n_rand=8000, box=250.0)
    e = np.geomspace(0.2, 40.0, 21)
    check_case("mono-open-log-auto-%g" % cell, d, None, cute.BIN_MONO, e, cell=cell)
    check_case("mono-open-log-cross-%g" % cell, d, r, cute.BIN_MONO, e, cell=cell)


def test_rmu_z_dd_dr_rr():
    d, r = catalogs.clustered_box_1e6(n_centres=150, per_blob=40, n_rand=15000, box=300.0)
    re_, me = np.linspace(0, 40, 9), np.linspace(0, 1, 11)
    check_case("rmu-dd", d, None, cute.BIN_RMU, re_, me)
    check_case("rmu-dr", d, r, cute.BIN_RMU, re_, me)
    check_case("rmu-rr", r, None, cute.BIN_RMU, re_, me)


def test_rmu_z_partial_mu_range_and_rmin():
    d, r = catalogs.clustered_box_1e6(n_centres=100, per_blob=30, n_rand=6000, box=200.0)
    check_case("rmu-partial", d, r, cute.BIN_RMU, np.linspace(2, 30, 8), np.linspace(0.1, 0.9, 9))


def test_rmu_midpoint_and_sigmapi_lightcone():
    d, r = catalogs.lightcone_3e6(n_data=6000, n_rand=9000, ra_max_deg=5.0, dec_max_deg=4.0)
    e = np.linspace(0, 40, 21)
    check_case("rmu-mid-dd", d, None, cute.BIN_RMU, e, np.linspace(0, 1, 11), los=cute.LOS_MIDPOINT)
    check_case("rmu-mid-dr", d, r, cute.BIN_RMU, e, np.linspace(0, 1, 11), los=cute.LOS_MIDPOINT)
    check_case("sigmapi-dd", d, None, cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
    check_case("sigmapi-dr", d, r, cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)


@pytest.mark.parametrize("centre", [(180.0, 0.0), (0.0, 10.0), (45.0, 89.0), (300.0, -88.5)])
def test_theta_caps(centre):
    """Equatorial cap, a cap straddling RA = 0 and caps around both poles."""
    d, r = catalogs.angular_cap_1e7(n_centres=60, per_blob=50, n_rand=9000, half_angle_deg=3.0,
                            centre=centre)
    e = np.deg2rad(np.geomspace(0.001, 2.0, 16))
    check_case("theta-dd-%s" % (centre,), d, None, cute.BIN_THETA, e, geom=cute.GEOM_SPHERE)
    check_case("theta-dr-%s" % (centre,), d, r, cute.BIN_THETA, e, geom=cute.GEOM_SPHERE)


def test_theta_linear_bins_large_angles():
    g = np.random.Generator(np.random.PCG64(7))
    v = g.normal(size=(5000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    e = np.deg2rad(np.linspace(0, 30, 13))
    check_case("theta-fullsky-lin", v, None, cute.BIN_THETA, e, geom=cute.GEOM_SPHERE)


def test_theta_axis_vectors_on_the_right_angle_edge():
    """Copies of the six axis unit vectors: their pairs lie at exactly 0, 90
    or 180 degrees, and 90 degrees is a bin edge, so FP32_EDGE must re-test
    them and decide each as FP64 and the oracle do; random unit vectors fill
    the other bins."""
    g = np.random.Generator(np.random.PCG64(31))
    axes = np.concatenate([np.eye(3), -np.eye(3)])
    v = g.normal(size=(2000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    pts = np.concatenate([np.repeat(axes, 40, axis=0), v])
    e = np.deg2rad(np.array([0.0, 30.0, 60.0, 90.0, 120.0]))
    check_case("theta-axis-ties", pts, None, cute.BIN_THETA, e, geom=cute.GEOM_SPHERE)
    check_case("theta-axis-ties-cross", pts[:240], v[:500], cute.BIN_THETA, e, geom=cute.GEOM_SPHERE)


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_empty_and_single_point_catalogs():
    e = np.linspace(0, 10, 6)
    bn = cute.Binning(cute.BIN_MONO, e)
    empty = np.zeros((0, 3))
    one = np.array([[1.0, 2.0, 3.0]])
    some = catalogs.uniform_box(500, 20.0, seed=3).stacked()
    for prec in EXACT + [cute.PREC_FP32_ONLY]:
        say("case empty prec", prec)
        assert gpu_counts(empty, None, bn, prec, cute.GEOM_BOX_OPEN).sum() == 0
        assert gpu_counts(one, None, bn, prec, cute.GEOM_BOX_OPEN).sum() == 0
        assert gpu_counts(empty, some, bn, prec, cute.GEOM_BOX_OPEN).sum() == 0
        assert gpu_counts(some, empty, bn, prec, cute.GEOM_BOX_OPEN).sum() == 0
        got = gpu_counts(one, some, bn, prec, cute.GEOM_BOX_OPEN)
        want = oracle.count_pairs(one, some, obin(cute.BIN_MONO, e)).reshape(-1)
        np.testing.assert_array_equal(got, want)


def test_duplicates_and_zero_separation():
    pts = np.repeat(np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 8.0]]), 70, axis=0)
    check_case("dups-mono", pts, None, cute.BIN_MONO, [0.0, 1.0, 2.0, 4.0])
    check_case("dups-rmu", pts, None, cute.BIN_RMU, [0.0, 1.0, 2.0, 4.0], [0.0, 0.5, 1.0])
    check_case("dups-rmu-cross", pts, pts[::3], cute.BIN_RMU, [0.0, 1.0, 2.0, 4.0], [0.0, 0.5, 1.0])


def test_dyadic_lattice_on_edges():
    """Lattice points give many pairs exactly on r and mu edges; every FP64
    operation is exact there, so FP32_EDGE must resolve each one like FP64."""
    g = np.random.Generator(np.random.PCG64(9))
    pts = g.integers(0, 24, size=(3000, 3)).astype(np.float64) * 0.5
    check_case("lattice-mono", pts, None, cute.BIN_MONO, np.arange(0, 9) * 0.5)
    check_case("lattice-rmu", pts, None, cute.BIN_RMU, np.arange(0, 9) * 0.5,
               np.array([0.0, 0.25, 0.5, 0.75, 1.0]))
    check_case("lattice-mono-periodic", pts, None, cute.BIN_MONO, np.arange(0, 9) * 0.5,
               geom=cute.GEOM_BOX_PERIODIC, L=12.0)


def test_dyadic_lattice_midpoint_on_edges():
    """Lattice points around the z axis, 100 away from the origin: for the
    pairs placed symmetrically about the axis the midpoint line of sight is
    exactly z, and pi = |dz| and sigma^2 = dx^2 + dy^2 fall on the sigma, pi,
    r and mu edges; the canonical FP64 predicates are exact there, so
    FP32_EDGE must resolve every tie as FP64 and the oracle do."""
    g = np.random.Generator(np.random.PCG64(19))
    pts = g.integers(-12, 12, size=(3000, 3)).astype(np.float64) * 0.5
    pts[:, 2] += 100.0
    e = np.arange(0, 9) * 0.5
    check_case("lattice-sigmapi", pts, None, cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
    check_case("lattice-rmu-mid", pts, None, cute.BIN_RMU, e, np.array([0.0, 0.25, 0.5, 0.75, 1.0]),
               los=cute.LOS_MIDPOINT)
    check_case("lattice-sigmapi-cross", pts[:1500], pts[1500:], cute.BIN_SIGMAPI, e, e,
               los=cute.LOS_MIDPOINT)


def test_periodic_pairs_across_faces():
    L = 100.0
    a = np.array([[0.0, 0.0, 0.0], [99.5, 0.25, 50.0], [50.0, 99.75, 0.5], [0.5, 0.5, 99.5]])
    b = catalogs.uniform_box(3000, L, seed=5).stacked()
    pts = np.concatenate([a, b])
    check_case("faces", pts, None, cute.BIN_MONO, np.linspace(0, 20, 11),
               geom=cute.GEOM_BOX_PERIODIC, L=L)


# ---------------------------------------------------------------------------
# Properties that hold at any size
# ---------------------------------------------------------------------------
def test_symmetry_and_fp32_only_bound():
    d, r = catalogs.clustered_box_1e6(n_centres=200, per_blob=50, n_rand=20000, box=400.0)
    bn = cute.Binning(cute.BIN_RMU, np.linspace(0, 50, 11), np.linspace(0, 1, 21))
    ga, gb = cute.build_grid(d, cute.GEOM_BOX_OPEN, r_max=50.0), cute.build_grid(r, cute.GEOM_BOX_OPEN, r_max=50.0)
    say("case symmetry")
    ab, st = cute.count_pairs(ga, gb, bn, cute.PREC_FP32_EDGE, with_stats=True)
    ba = cute.count_pairs(gb, ga, bn, cute.PREC_FP32_EDGE)
    np.testing.assert_array_equal(ab, ba)
    ab64 = cute.count_pairs(ga, gb, bn, cute.PREC_FP64)
    np.testing.assert_array_equal(ab, ab64)
    only = cute.count_pairs(ga, gb, bn, cute.PREC_FP32_ONLY).astype(np.int64)
    l1 = int(np.abs(only - ab.astype(np.int64)).sum())
    assert l1 <= 2 * st["flips"]
    assert st["retests"] >= st["flips"]
    say("retest fraction %.2e flips %d l1 %d" % (st["retests"] / max(1, st["pair_evals"]),
                                                 st["flips"], l1))


# ---------------------------------------------------------------------------
# Estimators and multipoles (host arithmetic in the library)
# ---------------------------------------------------------------------------
def test_estimators_match_exact_rationals():
    g = np.random.Generator(np.random.PCG64(11))
    nd, nr = 1_000_000, 2_000_000
    rr = g.integers(1, 10 ** 12, size=(8, 5)).astype(np.uint64)
    dd = (rr.astype(np.float64) * (nd * (nd - 1)) / (nr * (nr - 1)) * (1 + g.normal(0, 1e-4, rr.shape)))
    dd = np.rint(dd).astype(np.uint64)
    dr = (rr.astype(np.float64) * (2 * nd) / (nr - 1) * (1 + g.normal(0, 1e-4, rr.shape)))
    dr = np.rint(dr).astype(np.uint64)
    rr[0, 0] = 0
    bn = cute.Binning(cute.BIN_RMU, np.linspace(0, 40, 9), np.linspace(0, 1, 6))
    for e, ref in ((cute.EST_NATURAL, est.natural(dd, rr, nd, nr)),
                   (cute.EST_LS, est.landy_szalay(dd, dr, rr, nd, nr))):
        got = cute.xi_estimate(e, dd, dr, rr, nd, nr, bn)
        assert math.isnan(got[0, 0]) and math.isnan(ref[0, 0])
        m = ~np.isnan(ref)
        rel = np.abs(got[m] - ref[m]) / np.maximum(np.abs(ref[m]), 1e-300)
        assert rel.max() <= 1e-12, rel.max()
    e = np.arange(31) * 5.0
    ddb = g.integers(10, 10 ** 6, size=30).astype(np.uint64)
    got = cute.xi_estimate(cute.EST_BOX, ddb, None, None, 20000, 0, cute.Binning(cute.BIN_MONO, e),
                           box_size=1000.0)
    ref = est.box(ddb, 20000, 1000.0, e)
    assert np.max(np.abs((1 + got) - (1 + ref)) / (1 + ref)) <= 1e-13


def test_multipoles_match_exact_rationals():
    g = np.random.Generator(np.random.PCG64(12))
    mu = np.linspace(0, 1, 51)
    xi = g.normal(size=(40, 50))
    bn = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, mu)
    got = cute.xi_multipoles(xi, bn, (0, 2, 4))
    ref = est.multipoles(xi, mu, [0, 2, 4])
    for a, ell in enumerate((0, 2, 4)):
        w = est.multipole_weights_abs(mu, ell)
        scale = np.abs(xi) @ w
        assert np.all(np.abs(got[a] - ref[a]) <= 1e-12 * scale + 1e-300)


def test_tuned_grid_counts_match_oracle():
    """The grid tuner returns one of its (cell, tile) candidates with a time for
    each; counting with the chosen pair gives the oracle's counts."""
    d, _ = catalogs.clustered_box_1e6(n_centres=150, per_blob=40, n_rand=10, box=300.0)
    re_, me = np.linspace(0, 40, 9), np.linspace(0, 1, 11)
    bn = cute.Binning(cute.BIN_RMU, re_, me)
    cell, tile, times = cute.tune_grid(d, cute.GEOM_BOX_OPEN, bn)
    say("tuned grid", cell, tile, times)
    assert (cell, tile) in times and all(np.isfinite(v) and v > 0 for v in times.values())
    g = cute.build_grid(d, cute.GEOM_BOX_OPEN, r_max=40.0, cell_size=cell, tile_points=tile)
    np.testing.assert_array_equal(cute.count_pairs(g, None, bn, cute.PREC_FP32_EDGE),
                                  oracle.count_pairs(d, None, obin(cute.BIN_RMU, re_, me)))
    # explicit candidates in a periodic box, including small tiles
    u = catalogs.uniform_box(3000, 100.0, seed=5)
    e = np.linspace(0, 20, 11)
    mb = cute.Binning(cute.BIN_MONO, e)
    cell, tile, times = cute.tune_grid(u, cute.GEOM_BOX_PERIODIC, mb, box_size=100.0, r_max=20.0,
                                       cells=[5.0, 10.0], tiles=[1, 7, 64])
    assert set(times) == {(c, t) for c in (5.0, 10.0) for t in (1, 7, 64)}
    want = oracle.count_pairs(u, None, obin(cute.BIN_MONO, e, periodic=True, L=100.0))
    for t in (1, 7, 64):
        g = cute.build_grid(u, cute.GEOM_BOX_PERIODIC, box_size=100.0, r_max=20.0, cell_size=cell,
                            tile_points=t)
        for prec in EXACT:
            np.testing.assert_array_equal(cute.count_pairs(g, None, mb, prec), want)


@pytest.mark.parametrize("cell", [0.0, 1e9])
def test_table2_binnings(cell):
    """The binnings of the paper's Table 2 (256 linear r bins to 100, 256 log
    bins at 50 per decade, 64 x 64 sigma-pi, 256 linear theta bins to 30 deg)
    on DR of a small light-cone subset of its shape, with the cell list and
    with one cell holding every point (brute force)."""
    d, r = catalogs.lightcone_box(1500, seed=11), catalogs.lightcone_box(1500, seed=12)
    lin = np.linspace(0.0, 100.0, 257)
    check_case("t2-lin-%g" % cell, d, r, cute.BIN_MONO, lin, cell=cell)
    check_case("t2-log-%g" % cell, d, r, cute.BIN_MONO, 100.0 * 10.0 ** ((np.arange(257) - 256) / 50.0),
               cell=cell)
    sp = np.linspace(0.0, 100.0, 65)
    check_case("t2-sp-%g" % cell, d, r, cute.BIN_SIGMAPI, sp, sp, los=cute.LOS_MIDPOINT, cell=cell)
    du, ru = catalogs.unit_vectors(d), catalogs.unit_vectors(r)
    check_case("t2-theta-%g" % cell, du, ru, cute.BIN_THETA, np.deg2rad(np.linspace(0.0, 30.0, 257)),
               geom=cute.GEOM_SPHERE, cell=(1e9 if cell else 0.0))


@pytest.mark.parametrize("offset", [1e5, 3e6])
def test_far_from_the_origin_and_offset_grids(offset):
    """Catalogs far from the origin (large raw coordinates, small
    separations) and two grids whose boxes barely overlap (a large FP32 frame
    shift between them): FP64 and FP32_EDGE equal the oracle for r-mu (z line
    of sight) and sigma-pi (midpoint line of sight)."""
    d, r = catalogs.clustered_box_1e6(n_centres=80, per_blob=30, n_rand=3000, box=150.0)
    a = np.stack([d.x, d.y, d.z], axis=1) + offset
    b = np.stack([r.x, r.y, r.z], axis=1) + offset + np.array([120.0, 0.0, 0.0])
    check_case("far-rmu-auto-%g" % offset, a, None, cute.BIN_RMU, np.linspace(0, 30, 7),
               np.linspace(0, 1, 6))
    check_case("far-rmu-cross-%g" % offset, a, b, cute.BIN_RMU, np.linspace(0, 30, 7),
               np.linspace(0, 1, 6))
    e = np.linspace(0, 20, 6)
    check_case("far-sigmapi-cross-%g" % offset, a, b, cute.BIN_SIGMAPI, e, e,
               los=cute.LOS_MIDPOINT)


def test_rmu_fine_bins_far_apart_points():
    """r bins 5e-4 wide (r < 0.01) over a catalog 1000 across: the FP32
    coordinate error is a large part of a bin, so the count keeps the band
    tables for r and mu (cute_fp32_zlos_constants reports which). Close
    companions of spread-out anchors give pairs in every bin; FP64 and
    FP32_EDGE equal the oracle."""
    rng = np.random.default_rng(777)
    anchors = rng.uniform(0.0, 1000.0, (1500, 3))
    d = rng.normal(size=(1500, 3))
    d *= (rng.uniform(0.0, 0.011, 1500) / np.linalg.norm(d, axis=1))[:, None]
    pts = np.concatenate([anchors, anchors + d])
    check_case("rmu-fine-bins", pts, None, cute.BIN_RMU, np.linspace(0.0, 0.01, 21),
               np.linspace(0, 1, 11))


@pytest.mark.parametrize("flush", ["4096", "100000"])
def test_midpoint_histograms_moved_during_the_count(flush):
    """The midpoint kinds count in 32-bit LDS counters, moved to the global
    counts before they can wrap. A small flush threshold (a test hook; the
    count uses 2^30) makes the moves happen many times inside one count,
    while the other waves keep adding: single counts, a batch and the
    jackknife by regions still equal the oracle."""
    import os
    d, r = catalogs.clustered_box_1e6(n_centres=60, per_blob=40, n_rand=3000, box=200.0)
    a = np.stack([d.x, d.y, d.z], axis=1) + 1500.0
    b = np.stack([r.x, r.y, r.z], axis=1) + 1500.0
    e = np.linspace(0.0, 20.0, 11)
    os.environ["CUTE_TEST_H32_FLUSH"] = flush
    try:
        check_case("h32-sigmapi-auto-%s" % flush, a, None, cute.BIN_SIGMAPI, e, e,
                   los=cute.LOS_MIDPOINT)
        check_case("h32-sigmapi-cross-%s" % flush, a, b, cute.BIN_SIGMAPI, e, e,
                   los=cute.LOS_MIDPOINT)
        want = check_case("h32-rmumid-auto-%s" % flush, a, None, cute.BIN_RMU,
                          np.linspace(0.0, 30.0, 7), np.linspace(0, 1, 6), los=cute.LOS_MIDPOINT)
        bn = cute.Binning(cute.BIN_RMU, np.linspace(0.0, 30.0, 7), np.linspace(0, 1, 6),
                          los=cute.LOS_MIDPOINT)
        g = cute.build_grid(a, cute.GEOM_BOX_OPEN, r_max=30.0)
        items = [cute.BatchItem(g, None, bn), cute.BatchItem(g, None, bn)]
        reg = (a[:, 0] > np.median(a[:, 0])).astype(np.int32) + 2 * (a[:, 1] > np.median(a[:, 1]))
        ob = obin(cute.BIN_RMU, np.linspace(0.0, 30.0, 7), np.linspace(0, 1, 6), cute.LOS_MIDPOINT)
        wt, wj = oracle.count_jackknife(a, reg, 4, ob)
        for prec in EXACT:
            say("case h32 batch prec %d flush %s" % (prec, flush))
            got = cute.count_pairs_batched(items, prec)
            for x in got:
                np.testing.assert_array_equal(x.reshape(bn.shape), want)
            say("case h32 jackknife prec %d flush %s" % (prec, flush))
            tot, jack = cute.count_jackknife(g, reg, 4, bn, prec)
            np.testing.assert_array_equal(tot.reshape(-1), wt.reshape(-1))
            np.testing.assert_array_equal(jack.reshape(4, -1), wj.reshape(4, -1))
        g.close()
    finally:
        del os.environ["CUTE_TEST_H32_FLUSH"]


def test_periodic_rmax_close_to_half_box():
    """r_max = 0.49 L in a periodic box: every pair is still counted once
    (minimum image), against the oracle. Closer to L/2 a tile and its reach
    would need more cells than a grid may have: a clean CUTE_E_INVALID_ARG."""
    L = 200.0
    a = catalogs.mixed_periodic(3000, L, seed=131)
    e = np.linspace(0.0, 0.49 * L, 12)
    check_case("periodic-0.49L", a, None, cute.BIN_MONO, e, geom=cute.GEOM_BOX_PERIODIC, L=L)
    g = cute.build_grid(a, cute.GEOM_BOX_PERIODIC, box_size=L, r_max=0.4995 * L)
    with pytest.raises(cute.CuteError) as ex:
        cute.count_pairs(g, None, cute.Binning(cute.BIN_MONO, np.linspace(0.0, 0.4995 * L, 5)))
    assert ex.value.status == cute.E_INVALID_ARG


def test_concurrent_counts_on_two_streams():
    """One grid counted from two host threads, each on its own stream, with
    different binnings and precisions: every result equals the serial one."""
    import threading

    import torch
    d, r = catalogs.clustered_box_1e6(n_centres=150, per_blob=40, n_rand=8000, box=300.0)
    gd = cute.build_grid(d, cute.GEOM_BOX_OPEN, r_max=40.0)
    gr = cute.build_grid(r, cute.GEOM_BOX_OPEN, r_max=40.0)
    jobs = [(gd, None, cute.Binning(cute.BIN_RMU, np.linspace(0, 40, 9), np.linspace(0, 1, 11)),
             cute.PREC_FP32_EDGE),
            (gd, gr, cute.Binning(cute.BIN_MONO, np.geomspace(0.5, 40.0, 13)), cute.PREC_FP64),
            (gr, None, cute.Binning(cute.BIN_MONO, np.linspace(0, 40, 21)), cute.PREC_FP32_EDGE),
            (gd, gr, cute.Binning(cute.BIN_RMU, np.linspace(0, 40, 9), np.linspace(0, 1, 11)),
             cute.PREC_FP32_EDGE)]
    want = [cute.count_pairs(a, b, bn, p) for a, b, bn, p in jobs]
    got = [[None] * len(jobs) for _ in range(2)]
    errors = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            for rep in range(3):
                for k in (range(len(jobs)) if t == 0 else reversed(range(len(jobs)))):
                    a, b, bn, p = jobs[k]
                    got[t][k] = cute.count_pairs(a, b, bn, p, stream=s)
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for t in range(2):
        for k in range(len(jobs)):
            np.testing.assert_array_equal(got[t][k], want[k], err_msg="thread %d job %d" % (t, k))
