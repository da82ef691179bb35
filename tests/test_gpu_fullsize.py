"""Parity at the full sizes of the r-mu, light-cone (sigma-pi), angular and
batched workloads, against counts the CPU oracle computed at those sizes.

* r-mu (1e6 clustered data, 2e6 randoms): the full DD, DR and RR, and the
  Landy-Szalay estimator and multipoles built from them.
* sigma-pi light cone (3e6 data, 6e6 randoms): the full DD, DR and RR.
* batched (256 periodic mocks and the 100 jackknife catalogs of a 1e6-point
  base, monopole and r-mu binnings): every item of the batch and every
  leave-one-region-out count.
* angular cap (1e7 clustered data, 2e7 randoms): the oracle cannot count
  these whole (about 1e14 pair visits), so the check is sampled outputs plus
  properties that hold at any size. The sampled rows are the cross counts of
  1024 data and 1024 random points (768 random blob members or randoms, 256
  at the cap edge) against the whole data and random catalogs, counted
  through the full-size grids (every other point masked out), so that the
  full-size stencil, tiling and FP32 frame decide them. The full DD, DR and
  RR must then give the same counts in FP32_EDGE and FP64.
Expected values come from tests/golden/make_golden.py (oracle only); each
record holds the SHA-256 of its inputs, which the tests check first. FP64 and
FP32_EDGE must both equal them bit for bit."""
import json
import os
import sys

import numpy as np
import pytest

import catalogs
import paper_1210_1833_amd as cute

pytestmark = pytest.mark.gpu

EXACT = [cute.PREC_FP64, cute.PREC_FP32_EDGE]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.fail("missing golden counts %s (tests/golden/make_golden.py %s)" % (path, name))
    with open(path) as f:
        return json.load(f)


def dev_xyz(cat):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for v in (cat.x, cat.y, cat.z)]


def dgrid(cat, geom, r_max, L=0.0):
    return cute.build_grid(dev_xyz(cat), geom, box_size=L, r_max=r_max)


def counts_of(rec, shape):
    return np.array(rec["counts"], dtype=np.uint64).reshape(shape)


def check_full(ga, gb, bn, want, name):
    """FP64 and FP32_EDGE counts equal the oracle's; returns the FP32_EDGE stats."""
    st32 = None
    for prec in EXACT:
        say("%s prec %d" % (name, prec))
        got, st = cute.count_pairs(ga, gb, bn, prec, with_stats=True)
        np.testing.assert_array_equal(got, want, err_msg="%s prec %d" % (name, prec))
        assert st["pairs_in_range"] == int(want.sum())
        say("  %d pairs in range, %d evaluations, %d re-tests, %.1f ms"
            % (st["pairs_in_range"], st["pair_evals"], st["retests"], st["ms_count"]))
        if prec == cute.PREC_FP32_EDGE:
            st32 = st
    return st32


def test_rmu_dr_rr_full_size_and_estimators():
    """The r-mu workload beyond DD: the full DR (1e6 x 2e6) and RR (2e6) equal
    the oracle's; Landy-Szalay xi(r, mu) and its multipoles from the full
    counts agree with the oracle's exact-rational estimators to 1e-12."""
    from oracle import estimators as est
    d, r = catalogs.clustered_box_1e6()
    gdd, gdr, grr = (golden("clustered_1e6_%s_rmu" % k) for k in ("dd", "dr", "rr"))
    assert catalogs.sha256_of(d) == gdd["sha256"] == gdr["sha256_data"]
    assert catalogs.sha256_of(r) == gdr["sha256_randoms"] == grr["sha256_randoms"]
    e1, e2 = np.array(gdr["r_edges"]), np.array(gdr["mu_edges"])
    bn = cute.Binning(cute.BIN_RMU, e1, e2, los=cute.LOS_Z)
    dd, dr, rr = (counts_of(g, bn.shape) for g in (gdd, gdr, grr))
    gd = dgrid(d, cute.GEOM_BOX_OPEN, 200.0)
    gr = dgrid(r, cute.GEOM_BOX_OPEN, 200.0)
    check_full(gd, gr, bn, dr, "r-mu full size DR")
    check_full(gr, None, bn, rr, "r-mu full size RR")
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


@pytest.mark.parametrize("kind", ["dd", "dr", "rr"])
def test_sigmapi_lightcone_full_size(kind):
    """3e6 data and 6e6 randoms in the light cone; sigma and pi edges 2k Mpc/h
    (k <= 75), midpoint line of sight: the full count equals the oracle's."""
    g = golden("lightcone_3e6_%s_sigmapi" % kind)
    say("generating the light-cone catalogs")
    d, r = catalogs.lightcone_3e6()
    assert catalogs.sha256_of(d) == g["sha256_data"]
    assert catalogs.sha256_of(r) == g["sha256_randoms"]
    e = np.array(g["edges"])
    bn = cute.Binning(cute.BIN_SIGMAPI, e, e, los=cute.LOS_MIDPOINT)
    rmax = float(np.hypot(e[-1], e[-1])) * (1.0 + 1e-12)
    a, b = {"dd": (d, None), "dr": (d, r), "rr": (r, None)}[kind]
    ga = dgrid(a, cute.GEOM_BOX_OPEN, rmax)
    gb = None if b is None else dgrid(b, cute.GEOM_BOX_OPEN, rmax)
    st = check_full(ga, gb, bn, counts_of(g, bn.shape), "sigma-pi full size %s" % kind.upper())
    assert st["pairs_in_range"] > 0


@pytest.fixture(scope="module")
def cap():
    """The angular workload at full size: 1e7 clustered data and 2e7 randoms
    in a 5000 sq-deg cap, 30 log bins of theta in [0.001, 10] degrees, two
    grids of each catalog (the second is the partner of a cross count of a
    catalog with itself)."""
    g = golden("angular_cap_1e7_rows")
    say("generating the angular catalogs")
    d, r = catalogs.angular_cap_1e7()
    assert catalogs.sha256_of(d) == g["sha256_data"]
    assert catalogs.sha256_of(r) == g["sha256_randoms"]
    e = np.array(g["theta_edges_rad"])
    bn = cute.Binning(cute.BIN_THETA, e)
    say("building the four angular grids")
    grids = {"d": dgrid(d, cute.GEOM_SPHERE, e[-1]), "d2": dgrid(d, cute.GEOM_SPHERE, e[-1]),
             "r": dgrid(r, cute.GEOM_SPHERE, e[-1]), "r2": dgrid(r, cute.GEOM_SPHERE, e[-1])}
    yield g, len(d), len(r), bn, grids
    for v in grids.values():
        v.close()


def test_theta_cap_sampled_rows_through_full_size_grids(cap):
    """Rows of 1024 sampled data points and 1024 sampled randoms against the
    whole data and random catalogs, counted through the full-size grids with
    every other home point masked out, equal the oracle's rows."""
    import torch
    g, nd, nr, bn, G = cap

    def keep_only(n, idx):
        m = torch.ones(n, dtype=torch.uint8, device="cuda")
        m[torch.from_numpy(np.asarray(idx, dtype=np.int64)).to("cuda")] = 0
        return m

    md = keep_only(nd, g["sample_data_idx"])
    mr = keep_only(nr, g["sample_randoms_idx"])
    items = {"sd_x_d": cute.BatchItem(G["d"], G["d2"], bn, mask_a=md),
             "sd_x_r": cute.BatchItem(G["d"], G["r"], bn, mask_a=md),
             "sr_x_d": cute.BatchItem(G["r"], G["d"], bn, mask_a=mr),
             "sr_x_r": cute.BatchItem(G["r"], G["r2"], bn, mask_a=mr)}
    names = list(items)
    for prec in EXACT:
        say("theta full size: sampled rows through the full-size grids, prec %d" % prec)
        got = cute.count_pairs_batched([items[k] for k in names], prec)
        for k, c in zip(names, got):
            want = np.array(g["counts"][k], dtype=np.uint64)
            assert want.sum() > 0
            np.testing.assert_array_equal(c.reshape(-1), want, err_msg="%s prec %d" % (k, prec))


@pytest.mark.parametrize("kind", ["dd", "dr", "rr"])
def test_theta_cap_full_size_fp32_edge_equals_fp64(cap, kind):
    """The full DD (1e7), DR (1e7 x 2e7) and RR (2e7) of the angular workload:
    the FP32 path with its FP64 re-test gives the FP64 counts."""
    _, _, _, bn, G = cap
    ga, gb = {"dd": (G["d"], None), "dr": (G["d"], G["r"]), "rr": (G["r"], None)}[kind]
    say("theta full size: %s, FP32_EDGE" % kind.upper())
    c32, st = cute.count_pairs(ga, gb, bn, cute.PREC_FP32_EDGE, with_stats=True)
    say("  %d pairs in range, %d evaluations, %d re-tests, %.1f ms"
        % (st["pairs_in_range"], st["pair_evals"], st["retests"], st["ms_count"]))
    say("theta full size: %s, FP64" % kind.upper())
    c64, st64 = cute.count_pairs(ga, gb, bn, cute.PREC_FP64, with_stats=True)
    say("  %.1f ms" % st64["ms_count"])
    np.testing.assert_array_equal(c32, c64, err_msg=kind)
    assert st["pairs_in_range"] > 0


def test_batched_mocks_and_jackknife_full_size():
    """The batched workload at full size, in the benchmark's form: 256
    periodic mocks (2e4 .. 5e5 points) and the 100 jackknife catalogs of the
    1e6-point base (one 100 x 100 column of (x, y) masked each), every catalog
    with the monopole and the r-mu binnings, 712 items in one batch per
    precision; then all 100 jackknife counts again by region decomposition.
    Every count equals the oracle's."""
    import hashlib

    import torch
    g = golden("batched_mocks_256")
    npz_path = os.path.join(GOLDEN, g["counts_file"])
    with open(npz_path, "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == g["counts_file_sha256"]
    want = np.load(npz_path, allow_pickle=False)
    L = 1000.0
    say("generating the batched workload")
    mocks, base, region = catalogs.batched_mocks_256()
    h = hashlib.sha256()
    for m in mocks:
        h.update(catalogs.sha256_of(m).encode())
    assert h.hexdigest() == g["sha256_mocks"]
    assert catalogs.sha256_of(base) == g["sha256_base"]
    mono = cute.Binning(cute.BIN_MONO, np.array(g["mono_edges"]))
    rmu = cute.Binning(cute.BIN_RMU, np.array(g["r_edges"]), np.array(g["mu_edges"]),
                       los=cute.LOS_Z)
    gm = [dgrid(m, cute.GEOM_BOX_PERIODIC, 200.0, L) for m in mocks]
    gb = dgrid(base, cute.GEOM_BOX_PERIODIC, 200.0, L)
    reg = torch.from_numpy(region.astype(np.int32)).cuda()
    items = []
    for gk in gm:
        items += [cute.BatchItem(gk, None, mono), cute.BatchItem(gk, None, rmu)]
    for k in range(100):
        m = (reg == k).to(torch.uint8)
        items += [cute.BatchItem(gb, None, mono, mask_a=m), cute.BatchItem(gb, None, rmu, mask_a=m)]
    nm = len(gm)
    for prec in EXACT:
        say("full-size batch, prec %d, %d items" % (prec, len(items)))
        got, st = cute.count_pairs_batched(items, prec, with_stats=True)
        say("  %.1f ms, %d pair evaluations, %d re-tests"
            % (st["ms_count"], st["pair_evals"], st["retests"]))
        for k in range(nm):
            np.testing.assert_array_equal(got[2 * k].reshape(-1), want["mono"][k].reshape(-1),
                                          err_msg="mock %d monopole prec %d" % (k, prec))
            np.testing.assert_array_equal(got[2 * k + 1].reshape(-1), want["rmu"][k].reshape(-1),
                                          err_msg="mock %d r-mu prec %d" % (k, prec))
        for k in range(100):
            np.testing.assert_array_equal(got[2 * nm + 2 * k].reshape(-1),
                                          want["jk_mono"][k].reshape(-1),
                                          err_msg="jackknife %d monopole prec %d" % (k, prec))
            np.testing.assert_array_equal(got[2 * nm + 2 * k + 1].reshape(-1),
                                          want["jk_rmu"][k].reshape(-1),
                                          err_msg="jackknife %d r-mu prec %d" % (k, prec))
    reg_h = np.ascontiguousarray(region, dtype=np.int32)
    for name, bn_ in (("mono", mono), ("rmu", rmu)):
        for prec in EXACT:
            say("jackknife by regions, %s, prec %d" % (name, prec))
            total, jack = cute.count_jackknife(gb, reg_h, 100, bn_, prec)
            np.testing.assert_array_equal(total.reshape(-1), want["jk_total_" + name].reshape(-1))
            np.testing.assert_array_equal(jack.reshape(100, -1), want["jk_" + name].reshape(100, -1))
