"""Pins of the oracle's pixelised angular correlation (Sec. 3.4, angular
correlation function): the pixel rule against the geometry it defines, the
centres against their pixels, and the weighted counts against the unweighted
oracle on the expanded catalog, closed-form totals and a pure-Python brute
force."""
import numpy as np
import pytest

import oracle


def unit(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def test_ring_rule_at_exact_ring_boundaries():
    """cos(theta) boundaries of a power-of-two ring count are exact doubles:
    a point on a boundary opens the upper ring; z = 1 is in the last ring."""
    n_cth, n_phi = 16, 8
    z = -1.0 + 2.0 * np.arange(n_cth + 1) / n_cth
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    pts = np.stack([s, np.zeros_like(s), z], axis=1)
    ids = oracle.pixel_ids(pts, n_cth, n_phi)
    rings = ids // n_phi
    np.testing.assert_array_equal(rings, list(range(n_cth)) + [n_cth - 1])


def test_sector_rule_on_the_axes():
    """Points on the x and y axes lie on sector boundaries 0, n/4, n/2, 3n/4
    and open those sectors; poles go to sector 0."""
    n_cth, n_phi = 4, 32
    pts = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                   dtype=np.float64)
    ids = oracle.pixel_ids(pts, n_cth, n_phi)
    np.testing.assert_array_equal(ids % n_phi, [0, 8, 16, 24, 0, 0])
    np.testing.assert_array_equal(ids // n_phi, [2, 2, 2, 2, 3, 0])


def test_pixel_ids_match_the_angles():
    """Away from pixel boundaries the pixel is the one that contains the
    point's (cos theta, phi), computed here with numpy's arctan2."""
    n_cth, n_phi = 64, 96
    v = unit(20000, 11)
    ids = oracle.pixel_ids(v, n_cth, n_phi)
    t = (v[:, 2] + 1.0) * 0.5 * n_cth
    f = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi) * n_phi / (2 * np.pi)
    clear = (np.abs(t - np.round(t)) > 1e-9) & (np.abs(f - np.round(f)) > 1e-9)
    assert clear.mean() > 0.999
    want = np.floor(t).astype(np.int64) * n_phi + np.floor(f).astype(np.int64) % n_phi
    np.testing.assert_array_equal(ids[clear], want[clear])


def test_pixels_have_equal_area():
    """Ring widths in cos(theta) are equal and sectors equal in phi, so every
    pixel has area 4 pi / (n_cth n_phi): a large uniform sample fills the
    pixels evenly (chi-square within 5 sigma of its mean)."""
    n_cth, n_phi = 8, 16
    npix = n_cth * n_phi
    v = unit(400000, 12)
    c = np.bincount(oracle.pixel_ids(v, n_cth, n_phi), minlength=npix)
    e = len(v) / npix
    chi2 = ((c - e) ** 2 / e).sum()
    assert abs(chi2 - (npix - 1)) < 5 * np.sqrt(2 * (npix - 1))


def test_centres_lie_in_their_pixels():
    n_cth, n_phi = 32, 40
    ids = np.arange(n_cth * n_phi)
    x, y, z = oracle.pixel_centres(ids, n_cth, n_phi)
    np.testing.assert_allclose(x * x + y * y + z * z, 1.0, rtol=0, atol=1e-15)
    back = oracle.pixel_ids(np.stack([x, y, z], axis=1), n_cth, n_phi)
    np.testing.assert_array_equal(back, ids)
    # centre angles are the middle of the ring in cos(theta) and of the sector
    r, k = ids // n_phi, ids % n_phi
    np.testing.assert_allclose(z, -1.0 + (2 * r + 1) / n_cth, atol=1e-15)
    np.testing.assert_allclose(np.mod(np.arctan2(y, x), 2 * np.pi), 2 * np.pi * (k + 0.5) / n_phi,
                               atol=1e-12)


def test_pixel_map_conserves_objects():
    v = unit(5000, 13)
    m = oracle.pixel_map(v, 20, 30)
    assert m.counts.sum() == len(v)
    assert np.all(np.diff(m.ids) > 0) and np.all(m.counts > 0)


def expand(m):
    """The catalog that puts each object at its pixel centre."""
    rep = m.counts.astype(np.int64)
    return np.stack([np.repeat(m.x, rep), np.repeat(m.y, rep), np.repeat(m.z, rep)], axis=1)


@pytest.mark.parametrize("e0", [0.0, 0.05])
def test_weighted_counts_equal_counts_of_the_expanded_catalog(e0):
    """Each pair adds w_i w_j, and an autocorrelation adds w (w - 1) / 2 per
    pixel at zero separation: exactly the unweighted counts of the catalog
    in which every object sits at its pixel centre."""
    b = oracle.Binning(oracle.THETA, np.deg2rad(np.linspace(e0, 40.0, 17)))
    d = oracle.pixel_map(unit(3000, 14), 12, 24)
    r = oracle.pixel_map(unit(2500, 15), 12, 24)
    np.testing.assert_array_equal(oracle.count_weighted(d, d.counts, None, None, b),
                                  oracle.count_pairs(expand(d), None, b))
    np.testing.assert_array_equal(oracle.count_weighted(d, d.counts, r, r.counts, b),
                                  oracle.count_pairs(expand(d), expand(r), b))


def test_weighted_totals():
    """With bins covering [0, pi], the auto total is N (N - 1) / 2 object
    pairs and the cross total N_d N_r. An odd sector count leaves no two
    centres antipodal (antipodal centres can round to a chord of 2 or just
    above it, outside every half-open bin)."""
    b = oracle.Binning(oracle.THETA, np.array([0.0, 1.0, 2.0, np.pi]))
    d = oracle.pixel_map(unit(2000, 16), 10, 15)
    r = oracle.pixel_map(unit(1500, 17), 10, 15)
    assert int(oracle.count_weighted(d, d.counts, None, None, b).sum()) == 2000 * 1999 // 2
    assert int(oracle.count_weighted(d, d.counts, r, r.counts, b).sum()) == 2000 * 1500


def test_unit_weights_give_the_plain_counts():
    b = oracle.Binning(oracle.THETA, np.deg2rad(np.linspace(0.0, 60.0, 9)))
    v = unit(800, 18)
    w = np.ones(len(v), dtype=np.uint32)
    np.testing.assert_array_equal(oracle.count_weighted(v, w, None, None, b),
                                  oracle.count_pairs(v, None, b))


def test_weighted_counts_brute_force():
    """Pure Python: angles from arccos of the dot product, random weights."""
    rng = np.random.default_rng(19)
    a, b_ = unit(40, 20), unit(35, 21)
    wa = rng.integers(1, 9, len(a)).astype(np.uint32)
    wb = rng.integers(1, 9, len(b_)).astype(np.uint32)
    e = np.deg2rad(np.linspace(10.0, 170.0, 9))
    bn = oracle.Binning(oracle.THETA, e)
    want = np.zeros(8, dtype=np.uint64)
    for i in range(len(a)):
        for j in range(len(b_)):
            t = np.arccos(np.clip(a[i] @ b_[j], -1.0, 1.0))
            k = np.searchsorted(e, t, side="right") - 1
            if 0 <= k < 8:
                want[k] += int(wa[i]) * int(wb[j])
    np.testing.assert_array_equal(oracle.count_weighted(a, wa, b_, wb, bn), want)


def test_pixel_counts_approach_object_counts_at_large_angles():
    """Moving objects to pixel centres shifts separations by at most a pixel
    diagonal: at separations far above the pixel size the pixel counts stay
    within a few percent of the object counts."""
    v = unit(6000, 22)
    m = oracle.pixel_map(v, 256, 512)  # pixels about 0.4 deg on a side
    b = oracle.Binning(oracle.THETA, np.deg2rad(np.array([10.0, 20.0, 40.0, 80.0])))
    got = oracle.count_weighted(m, m.counts, None, None, b).astype(float)
    want = oracle.count_pairs(v, None, b).astype(float)
    np.testing.assert_allclose(got, want, rtol=0.02)


def test_rejects_bad_pixelisations():
    v = unit(10, 23)
    with pytest.raises(ValueError):
        oracle.pixel_ids(v, 0, 16)
    with pytest.raises(ValueError):
        oracle.pixel_ids(v, 4, 4)
