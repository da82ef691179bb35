"""Pins of the oracle's radial correlation counts (Sec. 2.1, radial 2PCF;
Sec. 3.4): pairs closer than an angular aperture, binned by the difference
of their redshifts. Checked against a pure-Python brute force, the 1-D
histogram of all redshift differences (an aperture that admits every pair,
and objects on one line of sight), exact ties on dyadic edges, and the
monotonicity of the counts in the aperture."""
import numpy as np
import pytest

import oracle


def unit(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def hist_all_pairs(ra, rb, edges, auto):
    """Half-open histogram of |ra_i - rb_j| over all pairs (i < j if auto)."""
    d = np.abs(ra[:, None] - rb[None, :])
    if auto:
        d = d[np.triu_indices(len(ra), 1)]
    d = d.ravel()
    k = np.searchsorted(edges, d, side="right") - 1
    ok = (d >= edges[0]) & (d < edges[-1])
    return np.bincount(k[ok], minlength=len(edges) - 1).astype(np.uint64)


def test_brute_force_pure_python():
    a, b = unit(60, 1), unit(50, 2)
    rng = np.random.default_rng(3)
    ra, rb = rng.uniform(0.5, 0.6, 60), rng.uniform(0.5, 0.6, 50)
    ap = np.deg2rad(70.0)
    e = np.linspace(0.0, 0.08, 9)
    want = np.zeros(8, dtype=np.uint64)
    for i in range(60):
        for j in range(50):
            if np.arccos(np.clip(a[i] @ b[j], -1, 1)) < ap:
                dz = abs(ra[i] - rb[j])
                k = np.searchsorted(e, dz, side="right") - 1
                if 0 <= k < 8:
                    want[k] += 1
    np.testing.assert_array_equal(oracle.count_radial(a, ra, b, rb, ap, e), want)


def test_full_aperture_is_the_histogram_of_all_differences():
    """An aperture of pi admits every pair that is not antipodal (none here),
    so the counts are the plain histogram of |z_i - z_j|."""
    a = unit(700, 4)
    r = np.random.default_rng(5).uniform(0.0, 1.0, 700)
    e = np.linspace(0.0, 0.9, 31)
    np.testing.assert_array_equal(oracle.count_radial(a, r, None, None, np.pi, e),
                                  hist_all_pairs(r, r, e, True))


def test_one_line_of_sight():
    """Objects in one direction: every pair has zero angle and is counted,
    whatever the aperture."""
    n = 400
    d = np.tile(np.array([[0.6, 0.0, 0.8]]), (n, 1))
    rng = np.random.default_rng(6)
    ra = rng.uniform(0.4, 0.7, n)
    rb = rng.uniform(0.4, 0.7, n)
    e = np.linspace(0.0, 0.3, 16)
    np.testing.assert_array_equal(oracle.count_radial(d, ra, None, None, 1e-6, e),
                                  hist_all_pairs(ra, ra, e, True))
    np.testing.assert_array_equal(oracle.count_radial(d, ra, d, rb, 1e-6, e),
                                  hist_all_pairs(ra, rb, e, False))


def test_dyadic_ties_open_the_upper_bin():
    """Redshifts on a 1/64 grid and edges on a 1/16 grid: differences equal
    to an edge are exact and go to the bin that the edge opens; a difference
    equal to the last edge is not counted."""
    d = np.tile(np.array([[0.0, 0.0, 1.0]]), (5, 1))
    r = np.array([0.5, 0.5625, 0.625, 0.75, 0.8125])  # differences 1/16 .. 5/16
    e = np.arange(5) / 16.0                          # 0, 1/16, .., 4/16
    got = oracle.count_radial(d, r, None, None, 0.1, e)
    np.testing.assert_array_equal(got, hist_all_pairs(r, r, e, True))
    # 1/16 three times, 2/16 twice, 3/16 twice; the two differences of 4/16
    # equal the last edge and are left out
    np.testing.assert_array_equal(got, [0, 3, 2, 2])


def test_counts_grow_with_the_aperture():
    a = unit(1500, 7)
    r = np.random.default_rng(8).uniform(0.0, 0.2, 1500)
    e = np.linspace(0.0, 0.1, 11)
    prev = np.zeros(10, dtype=np.uint64)
    for deg in (2.0, 5.0, 10.0, 30.0):
        c = oracle.count_radial(a, r, None, None, np.deg2rad(deg), e)
        assert np.all(c >= prev)
        prev = c
    assert prev.sum() > 0


def test_aperture_boundary_is_strict():
    """Two objects exactly 90 degrees apart: counted for an aperture just
    above, not for one of 90 degrees (chord^2 = 2 = the threshold)."""
    p = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    r = np.array([0.1, 0.2])
    e = np.array([0.0, 1.0])
    assert oracle.count_radial(p, r, None, None, np.pi / 2 + 1e-9, e)[0] == 1
    c = 2.0 * np.sin(0.25 * np.pi)
    if c * c == 2.0:
        assert oracle.count_radial(p, r, None, None, np.pi / 2, e)[0] == 0


def test_rejects_bad_arguments():
    a = unit(3, 9)
    r = np.zeros(3)
    with pytest.raises(ValueError):
        oracle.count_radial(a, r, None, None, 0.0, [0.0, 1.0])
    with pytest.raises(ValueError):
        oracle.count_radial(a, r, None, None, 0.1, [0.0, 0.0])
    with pytest.raises(ValueError):
        oracle.count_radial(a, r[:2], None, None, 0.1, [0.0, 1.0])
