"""GPU parity of the radial correlation counts (Sec. 2.1, radial 2PCF; Sec.
3.4): pairs within an angular aperture binned by redshift difference, from
the HIP library (through the C ABI) against the oracle, bit-exact, on seeded
light-cone-like catalogs (clustered in angle and redshift), at several
apertures, with exact ties, empty inputs and the Table 2 catalog size."""
import sys

import numpy as np
import pytest

import catalogs
import oracle
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


def patch(n, seed, blobs=0, side_deg=18.0, sig_deg=0.2, sig_z=0.002):
    """Unit vectors in an RA x Dec patch [0, side]^2 and redshifts in
    [0.5, 0.6]: uniform, or in Gaussian blobs in angle and redshift."""
    rng = np.random.default_rng(seed)
    if blobs:
        ra0 = rng.uniform(0, side_deg, blobs)
        de0 = rng.uniform(0, side_deg, blobs)
        z0 = rng.uniform(0.5, 0.6, blobs)
        k = rng.integers(0, blobs, n)
        ra = ra0[k] + rng.normal(scale=sig_deg, size=n)
        de = np.clip(de0[k] + rng.normal(scale=sig_deg, size=n), -89.0, 89.0)
        z = z0[k] + rng.normal(scale=sig_z, size=n)
    else:
        ra = rng.uniform(0, side_deg, n)
        de = np.rad2deg(np.arcsin(rng.uniform(0.0, np.sin(np.deg2rad(side_deg)), n)))
        z = rng.uniform(0.5, 0.6, n)
    a, d = np.deg2rad(ra), np.deg2rad(de)
    v = np.stack([np.cos(d) * np.cos(a), np.cos(d) * np.sin(a), np.sin(d)], axis=1)
    return v, z


def grid(v, aperture):
    return cute.build_grid(v, cute.GEOM_SPHERE, r_max=aperture)


def check(d, zd, r, zr, aperture, edges):
    gd, gr = grid(d, aperture), grid(r, aperture)
    want_dd = oracle.count_radial(d, zd, None, None, aperture, edges)
    want_dr = oracle.count_radial(d, zd, r, zr, aperture, edges)
    assert want_dd.sum() > 0 and want_dr.sum() > 0
    np.testing.assert_array_equal(cute.count_radial(gd, zd, None, None, aperture, edges), want_dd)
    np.testing.assert_array_equal(cute.count_radial(gd, zd, gr, zr, aperture, edges), want_dr)
    np.testing.assert_array_equal(cute.count_radial(gr, zr, gd, zd, aperture, edges),
                                  oracle.count_radial(r, zr, d, zd, aperture, edges))


def test_radial_one_degree_clustered():
    """Aperture 1 deg, 50 bins of dz in [0, 0.05]: clustered data against
    uniform randoms."""
    d, zd = patch(20000, 1, blobs=400)
    r, zr = patch(30000, 2)
    say("radial, 1 deg aperture")
    check(d, zd, r, zr, np.deg2rad(1.0), np.linspace(0.0, 0.05, 51))


@pytest.mark.parametrize("ap_deg", [0.05, 5.0, 20.0])
def test_radial_apertures(ap_deg):
    """Narrow, wide and wider-than-the-cells apertures, log-spaced dz bins
    starting above zero."""
    d, zd = patch(6000, 3, blobs=100)
    r, zr = patch(6000, 4)
    say("radial, %g deg aperture" % ap_deg)
    check(d, zd, r, zr, np.deg2rad(ap_deg), 1e-4 * 10.0 ** (np.arange(31) / 10.0))


def test_radial_redshifts_on_device():
    import torch
    d, zd = patch(8000, 5, blobs=80)
    g = grid(d, np.deg2rad(1.0))
    e = np.linspace(0.0, 0.02, 21)
    host = cute.count_radial(g, zd, None, None, np.deg2rad(1.0), e)
    dev = cute.count_radial(g, torch.from_numpy(zd).cuda(), None, None, np.deg2rad(1.0), e)
    np.testing.assert_array_equal(host, dev)
    np.testing.assert_array_equal(host, oracle.count_radial(d, zd, None, None, np.deg2rad(1.0), e))


def test_radial_exact_ties_across_tiles():
    """40 directions with 100 objects each (many tiles share one point on the
    sphere), redshifts on a 1/1024 grid, edges on a 1/64 grid: differences
    equal to an edge open the upper bin."""
    rng = np.random.default_rng(6)
    dirs, _ = patch(40, 7, side_deg=4.0)
    v = np.repeat(dirs, 100, axis=0)
    z = rng.integers(512, 640, len(v)) / 1024.0
    e = np.arange(9) / 64.0
    g = grid(v, np.deg2rad(0.5))
    np.testing.assert_array_equal(cute.count_radial(g, z, None, None, np.deg2rad(0.5), e),
                                  oracle.count_radial(v, z, None, None, np.deg2rad(0.5), e))


def test_radial_empty_and_single():
    e = np.linspace(0.0, 0.1, 5)
    one, z1 = patch(1, 8)
    none = np.zeros((0, 3))
    g1, g0 = grid(one, 0.01), grid(none, 0.01)
    assert not cute.count_radial(g1, z1, None, None, 0.01, e).any()
    assert not cute.count_radial(g0, np.zeros(0), None, None, 0.01, e).any()
    assert not cute.count_radial(g1, z1, g0, np.zeros(0), 0.01, e).any()


def test_radial_table2_size():
    """The Table 2 light-cone subset (3e5 data, 3e5 randoms; directions from
    its positions, redshifts uniform in [0.5, 0.6]) with a 1 deg aperture:
    the DR rows of 64 sampled data objects equal the oracle's, and DR + RD
    agree."""
    d3, r3 = catalogs.table2()
    d, r = catalogs.unit_vectors(d3).stacked(), catalogs.unit_vectors(r3).stacked()
    rng = np.random.default_rng(9)
    zd, zr = rng.uniform(0.5, 0.6, len(d)), rng.uniform(0.5, 0.6, len(r))
    ap, e = np.deg2rad(1.0), np.linspace(0.0, 0.1, 101)
    gd, gr = grid(d, ap), grid(r, ap)
    dr, st = cute.count_radial(gd, zd, gr, zr, ap, e, with_stats=True)
    say("radial Table 2 size: %d pairs in range, %d evaluations, %.2f ms"
        % (st["pairs_in_range"], st["pair_evals"], st["ms_count"]))
    np.testing.assert_array_equal(dr, cute.count_radial(gr, zr, gd, zd, ap, e))
    idx = np.sort(rng.choice(len(d), 64, replace=False))
    gs = grid(d[idx], ap)
    np.testing.assert_array_equal(cute.count_radial(gs, zd[idx], gr, zr, ap, e),
                                  oracle.count_radial(d[idx], zd[idx], r, zr, ap, e))


def test_radial_rejections():
    v, z = patch(500, 10)
    g = grid(v, 0.02)
    e = np.linspace(0.0, 0.1, 5)
    box = cute.build_grid(np.random.default_rng(11).uniform(0, 10, (100, 3)), cute.GEOM_BOX_OPEN,
                          r_max=1.0)
    cases = [
        (lambda: cute.count_radial(box, np.zeros(100), None, None, 0.02, e), cute.E_INVALID_ARG),
        (lambda: cute.count_radial(g, z, None, None, 0.0, e), cute.E_INVALID_ARG),
        (lambda: cute.count_radial(g, z, None, None, 4.0, e), cute.E_INVALID_ARG),
        (lambda: cute.count_radial(g, z, None, None, 0.02, [0.1, 0.1]), cute.E_INVALID_ARG),
        (lambda: cute.count_radial(g, np.full(500, np.nan), None, None, 0.02, e), cute.E_INVALID_ARG),
        (lambda: cute.count_radial(cute.build_pixel_map(v, 64, 64, r_max=0.02),
                                   z, None, None, 0.02, e), cute.E_UNSUPPORTED),
    ]
    for f, status in cases:
        with pytest.raises(cute.CuteError) as ex:
            f()
        assert ex.value.status == status


def test_radial_counts_into_device_memory():
    """Counts written to a device tensor equal the host copy."""
    import torch
    d, zd = patch(5000, 12, blobs=50)
    g = grid(d, np.deg2rad(1.0))
    e = np.linspace(0.0, 0.02, 11)
    host = cute.count_radial(g, zd, None, None, np.deg2rad(1.0), e)
    out = torch.zeros(len(e) - 1, dtype=torch.int64, device="cuda")
    cute.count_radial(g, torch.from_numpy(zd).cuda(), None, None, np.deg2rad(1.0), e, out=out)
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.uint64), host)
