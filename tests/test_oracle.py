"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * a hand-worked example (golden fixture);
  * exact rational geometry on dyadic inputs, where every FP64 operation of
    the oracle is exact, so its counts must equal the exact-real counts;
  * the analytic expectation for uniform points (periodic box, full sphere),
    with the exact variance of the pair counts;
  * an independent classification through numpy's arccos for the angle;
  * identities of the pair count (symmetry, auto/cross, marginals, additivity)
    and the equality of the window-pruned and brute-force loops.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import catalogs
import oracle
from oracle import LOS_MID, LOS_Z, MONO, RMU, SIGMAPI, THETA, Binning

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Exact-real reference on dyadic inputs (written from the geometric
# definitions of Sec. 2.1: r = |s|, mu = |s.l|/(|s||l|), pi = r mu,
# sigma = sqrt(r^2 - pi^2); all squared and compared as rationals).
# ---------------------------------------------------------------------------
def _exact_bin(p, q, kind, e1, e2=None, los=LOS_Z, L=None):
    P = [Fraction(v) for v in p]
    Q = [Fraction(v) for v in q]
    s = [a - b for a, b in zip(P, Q)]
    if L is not None:
        Lq = Fraction(L)
        s = [v - Lq if v > Lq / 2 else (v + Lq if v < -Lq / 2 else v) for v in s]
    r2 = sum(v * v for v in s)
    E1 = [Fraction(v) ** 2 for v in e1]

    def last_le(t, v):
        k = None
        for i in range(len(t) - 1):
            if t[i] <= v:
                k = i
        return k

    if kind == MONO:
        if not (E1[0] <= r2 < E1[-1]):
            return -1
        return last_le(E1, r2)
    l = [a + b for a, b in zip(P, Q)]
    ll = sum(v * v for v in l)
    sl = sum(a * b for a, b in zip(s, l))
    if kind == RMU:
        if not (E1[0] <= r2 < E1[-1]):
            return -1
        ir = last_le(E1, r2)
        if los == LOS_Z:
            mu2 = Fraction(0) if r2 == 0 else s[2] ** 2 / r2
        else:
            mu2 = Fraction(0) if (r2 == 0 or ll == 0) else sl * sl / (r2 * ll)
        M = [Fraction(v) ** 2 for v in e2]
        if mu2 < M[0]:
            return -1
        if Fraction(e2[-1]) < 1 and mu2 >= M[-1]:
            return -1
        return ir * (len(e2) - 1) + max(j for j in range(len(e2) - 1) if M[j] <= mu2)
    if kind == SIGMAPI:
        if ll == 0:
            sig2, pi2 = r2, Fraction(0)
        else:
            pi2 = sl * sl / ll
            sig2 = r2 - pi2
        S = E1
        Pq = [Fraction(v) ** 2 for v in e2]
        if not (S[0] <= sig2 < S[-1]) or not (Pq[0] <= pi2 < Pq[-1]):
            return -1
        return last_le(S, sig2) * (len(e2) - 1) + last_le(Pq, pi2)
    raise ValueError(kind)


def _exact_counts(pts_a, pts_b, kind, e1, e2=None, los=LOS_Z, L=None):
    n1 = len(e1) - 1
    n2 = 1 if e2 is None else len(e2) - 1
    h = np.zeros(n1 * n2, dtype=np.uint64)
    if pts_b is None:
        for i in range(len(pts_a)):
            for j in range(i + 1, len(pts_a)):
                k = _exact_bin(pts_a[i], pts_a[j], kind, e1, e2, los, L)
                if k >= 0:
                    h[k] += 1
    else:
        for i in range(len(pts_a)):
            for j in range(len(pts_b)):
                k = _exact_bin(pts_a[i], pts_b[j], kind, e1, e2, los, L)
                if k >= 0:
                    h[k] += 1
    return h if e2 is None else h.reshape(n1, n2)


def _dyadic(n, seed, lo=0.0, hi=16.0, step=1.0 / 16):
    """Points on a 1/16 lattice: 8-bit coordinates keep every FP64 product and
    sum in the oracle exact, so its decisions equal the exact-real ones."""
    g = np.random.Generator(np.random.PCG64(seed))
    m = int(round((hi - lo) / step))
    return lo + g.integers(0, m, size=(n, 3)).astype(np.float64) * step


# ---------------------------------------------------------------------------
def test_golden_lattice_mono_and_rmu():
    with open(os.path.join(GOLDEN, "lattice_pairs.json")) as f:
        g = json.load(f)
    pts = np.array(g["points"], dtype=np.float64)
    h = oracle.count_pairs(pts, None, Binning(MONO, g["mono"]["edges"]))
    assert h.tolist() == g["mono"]["counts"]
    h = oracle.count_pairs(pts, None, Binning(MONO, g["mono_top_13"]["edges"]))
    assert h.tolist() == g["mono_top_13"]["counts"]
    r = g["rmu_z"]
    h = oracle.count_pairs(pts, None, Binning(RMU, r["r_edges"], r["mu_edges"], los=LOS_Z))
    assert h.tolist() == r["counts"]


@pytest.mark.parametrize("case", ["mono_open", "mono_periodic", "rmu_z", "rmu_mid",
                                  "sigmapi", "rmu_z_partial_mu", "mono_rmin"])
@pytest.mark.parametrize("mode", ["auto", "cross"])
def test_exact_on_dyadic_inputs(case, mode):
    a = _dyadic(70, 11)
    b = _dyadic(60, 12) if mode == "cross" else None
    # duplicates and shared planes exercise r = 0, mu = 0 and mu = 1
    a[5] = a[6]
    a[7, :2] = a[8, :2]
    a[9, 2] = a[10, 2]
    L = None
    if case == "mono_open":
        args = dict(kind=MONO, e1=[0, 0.5, 1.25, 2, 3.5, 4])
    elif case == "mono_rmin":
        args = dict(kind=MONO, e1=[0.25, 0.5, 1.25, 2, 3.5, 4])
    elif case == "mono_periodic":
        args = dict(kind=MONO, e1=[0, 0.5, 1.25, 2, 3.5, 4, 6])
        L = 16.0
    elif case == "rmu_z":
        args = dict(kind=RMU, e1=[0, 1, 2, 3, 4.5], e2=[0, 0.25, 0.5, 0.75, 1], los=LOS_Z)
    elif case == "rmu_z_partial_mu":
        args = dict(kind=RMU, e1=[0, 1, 2, 3, 4.5], e2=[0.125, 0.25, 0.5, 0.75], los=LOS_Z)
    elif case == "rmu_mid":
        args = dict(kind=RMU, e1=[0, 1, 2, 3, 4.5], e2=[0, 0.25, 0.5, 0.75, 1], los=LOS_MID)
    else:
        args = dict(kind=SIGMAPI, e1=[0, 0.5, 1, 2, 3], e2=[0, 0.5, 1, 1.5, 2.5], los=LOS_MID)
    if case in ("rmu_mid", "sigmapi"):
        # points on both sides of the observer so that l = p + q can vanish
        a = a - 8.0
        if b is not None:
            b = b - 8.0
        a[11] = -a[12]
    want = _exact_counts(a, b, args["kind"], args["e1"], args.get("e2"), args.get("los", LOS_Z), L)
    bn = Binning(args["kind"], args["e1"], args.get("e2"), los=args.get("los", LOS_Z),
                 periodic=L is not None, L=L or 0.0)
    got = oracle.count_pairs(a, b, bn)
    np.testing.assert_array_equal(got.reshape(want.shape), want)
    # the x-window prune must give the same counts
    got_w = oracle.count_pairs(a, b, bn, prune=True)
    np.testing.assert_array_equal(got_w, got)


def test_edge_cases_single_pairs():
    b = Binning(MONO, [0, 5, 10, 150])
    assert oracle.classify([0, 0, 0], [3, 4, 0], b) == 1        # r = 5 exactly: bin 1
    assert oracle.classify([0, 0, 0], [90, 120, 0], b) == -1    # r = 150: excluded
    assert oracle.classify([1, 2, 3], [1, 2, 3], b) == 0        # r = 0: first bin
    bp = Binning(MONO, [0, 5, 10, 150], periodic=True, L=1000.0)
    assert oracle.classify([999, 0, 0], [4, 0, 0], bp) == 1      # wraps to r = 5
    assert oracle.classify([0.5, 0, 0], [999.5, 0, 0], bp) == 0  # wraps to r = 1
    rmu = Binning(RMU, [0, 5, 10], [0, 0.5, 1], los=LOS_Z)
    assert oracle.classify([0, 0, 0], [0, 0, 5], rmu) == 1 * 2 + 1   # mu = 1: last bin
    assert oracle.classify([0, 0, 0], [5, 0, 0], rmu) == 1 * 2 + 0   # mu = 0
    assert oracle.classify([2, 2, 2], [2, 2, 2], rmu) == 0           # r = 0: mu bin 0
    # 3-4-5 triangle with dz = 3: mu = 0.6, the edge fl(0.6) lies below 0.6
    rmu6 = Binning(RMU, [0, 10], [0, 0.6, 1], los=LOS_Z)
    assert oracle.classify([0, 0, 0], [4, 0, 3], rmu6) == 1
    # midpoint line of sight: a radial pair has sigma = 0, pi = |a - b|
    sp = Binning(SIGMAPI, [0, 1, 2, 4], [0, 2, 4, 8], los=LOS_MID)
    assert oracle.classify([0, 0, 100], [0, 0, 103], sp) == 0 * 3 + 1
    # equidistant from the observer: s is perpendicular to l, pi = 0, sigma = r
    assert oracle.classify([1.5, 0, 100], [-1.5, 0, 100], sp) == 2 * 3 + 0
    # l = 0 (points opposite the observer): pi := 0, sigma := r
    assert oracle.classify([0.75, 0, 0], [-0.75, 0, 0], sp) == 1 * 3 + 0
    # theta: orthogonal unit vectors are 90 degrees apart (chord^2 = 2)
    th = Binning(THETA, np.deg2rad([0, 45, 90, 135]))
    assert oracle.classify([1, 0, 0], [0, 1, 0], th) == 2
    assert oracle.classify([1, 0, 0], [0, 0, -1], th) == 2
    assert oracle.classify([1, 0, 0], [1, 0, 0], th) == 0


def test_periodic_uniform_matches_analytic_rr():
    """Uniform points in a periodic box: E[DD_k] = C(N,2) V_k/L^3 and the pair
    indicators are pairwise uncorrelated, so Var = C(N,2) p_k (1 - p_k)."""
    cat = catalogs.periodic_uniform_2e4()
    n, L = len(cat), 1000.0
    edges = np.arange(31) * 5.0
    h = oracle.count_pairs(cat, None, Binning(MONO, edges, periodic=True, L=L), prune=True)
    npairs = n * (n - 1) / 2
    p = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3) / L ** 3
    mean = npairs * p
    sd = np.sqrt(npairs * p * (1 - p))
    z = (h.astype(np.float64) - mean) / sd
    assert np.all(np.abs(z) < 5), z
    chi2 = float(np.sum(z * z))
    assert stats.chi2.sf(chi2, len(p)) > 1e-6
    # the oracle's total must also be consistent with the total in-range probability
    ptot = p.sum()
    assert abs(h.sum() - npairs * ptot) < 5 * math.sqrt(npairs * ptot)


def test_full_sphere_uniform_matches_analytic_theta():
    """Uniform unit vectors: P(theta in [t_k, t_{k+1})) = (cos t_k - cos t_{k+1})/2."""
    g = np.random.Generator(np.random.PCG64(77))
    v = g.normal(size=(4000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    edges = np.deg2rad(np.linspace(0, 60, 16))
    h = oracle.count_pairs(v, None, Binning(THETA, edges))
    npairs = 4000 * 3999 / 2
    p = (np.cos(edges[:-1]) - np.cos(edges[1:])) / 2
    z = (h - npairs * p) / np.sqrt(npairs * p * (1 - p))
    # pairs of a uniform sample are not independent for the sphere beyond
    # pairwise, but the variance formula still holds pairwise (rotation
    # invariance), so the z-scores are standard
    assert np.all(np.abs(z) < 5), z


def test_theta_matches_arccos_classification():
    """Chord thresholds give the same bins as theta = arccos(n1 . n2) away
    from the edges (numpy's arccos is an independent route to the angle)."""
    c = catalogs.cap_uniform(150, 12.0, 30.0, 20.0, seed=5)
    v = c.stacked()
    edges = np.deg2rad(np.geomspace(0.05, 15.0, 13))
    bn = Binning(THETA, edges)
    checked = 0
    for i in range(len(v)):
        for j in range(i + 1, len(v)):
            cross = np.linalg.norm(np.cross(v[i], v[j]))
            theta = math.atan2(cross, float(np.dot(v[i], v[j])))
            if np.min(np.abs(theta - edges)) < 1e-9:
                continue
            k = int(np.searchsorted(edges, theta, side="right")) - 1
            want = k if 0 <= k < len(edges) - 1 else -1
            assert oracle.classify(v[i], v[j], bn) == want
            checked += 1
    assert checked > 10000


def _small_binnings(L=None):
    out = [Binning(MONO, np.linspace(0, 12, 13), periodic=L is not None, L=L or 0.0),
           Binning(RMU, np.linspace(0, 12, 7), np.linspace(0, 1, 6), los=LOS_Z,
                   periodic=L is not None, L=L or 0.0)]
    if L is None:
        out.append(Binning(RMU, np.linspace(0, 12, 7), np.linspace(0, 1, 6), los=LOS_MID))
        out.append(Binning(SIGMAPI, np.linspace(0, 9, 10), np.linspace(0, 9, 7), los=LOS_MID))
    return out


@pytest.mark.parametrize("periodic", [False, True])
def test_symmetry_and_auto_cross_identity(periodic):
    L = 60.0 if periodic else None
    a = catalogs.uniform_box(300, 60.0, seed=31)
    b = catalogs.uniform_box(250, 60.0, seed=32)
    for bn in _small_binnings(L):
        ab = oracle.count_pairs(a, b, bn)
        ba = oracle.count_pairs(b, a, bn)
        np.testing.assert_array_equal(ab, ba)                        # DR(A,B) == DR(B,A)
        aa = oracle.count_pairs(a, a, bn)
        auto = oracle.count_pairs(a, None, bn)
        expect = 2 * auto.astype(np.int64)
        expect.reshape(-1)[0] += len(a)                              # self pairs: r = 0, bin 0
        np.testing.assert_array_equal(aa.astype(np.int64), expect)


def test_rmu_marginal_equals_mono():
    d, r = catalogs.clustered_box_1e6(n_centres=40, per_blob=25, n_rand=800, box=120.0)
    re = np.linspace(0, 20, 9)
    mono = oracle.count_pairs(d, None, Binning(MONO, re))
    for los in (LOS_Z, LOS_MID):
        rmu = oracle.count_pairs(d, None, Binning(RMU, re, np.linspace(0, 1, 11), los=los))
        np.testing.assert_array_equal(rmu.sum(axis=1), mono)
    mono_x = oracle.count_pairs(d, r, Binning(MONO, re))
    rmu_x = oracle.count_pairs(d, r, Binning(RMU, re, np.linspace(0, 1, 11), los=LOS_Z))
    np.testing.assert_array_equal(rmu_x.sum(axis=1), mono_x)


def test_additivity_of_union():
    a = catalogs.uniform_box(200, 40.0, seed=41)
    b = catalogs.uniform_box(170, 40.0, seed=42)
    u = catalogs.Catalog(np.concatenate([a.x, b.x]), np.concatenate([a.y, b.y]),
                         np.concatenate([a.z, b.z]))
    for bn in _small_binnings():
        lhs = oracle.count_pairs(u, None, bn).astype(np.int64)
        rhs = (oracle.count_pairs(a, None, bn).astype(np.int64)
               + oracle.count_pairs(b, None, bn).astype(np.int64)
               + oracle.count_pairs(a, b, bn).astype(np.int64))
        np.testing.assert_array_equal(lhs, rhs)


@pytest.mark.parametrize("kind", ["mono_periodic", "rmu_open", "sigmapi", "theta"])
def test_window_prune_equals_brute_force(kind):
    if kind == "mono_periodic":
        a = catalogs.mixed_periodic(3000, 100.0, seed=51)
        b = catalogs.uniform_box(2000, 100.0, seed=52)
        bn = Binning(MONO, np.linspace(0, 30, 16), periodic=True, L=100.0)
    elif kind == "rmu_open":
        a, b = catalogs.clustered_box_1e6(n_centres=30, per_blob=100, n_rand=3000, box=200.0)
        bn = Binning(RMU, np.linspace(0, 25, 6), np.linspace(0, 1, 11), los=LOS_Z)
    elif kind == "sigmapi":
        a, b = catalogs.lightcone_3e6(n_data=2000, n_rand=2500, ra_max_deg=4.0, dec_max_deg=3.0)
        bn = Binning(SIGMAPI, np.linspace(0, 30, 16), np.linspace(0, 30, 16), los=LOS_MID)
    else:
        a, b = catalogs.angular_cap_1e7(n_centres=30, per_blob=50, n_rand=2500, half_angle_deg=5.0)
        bn = Binning(THETA, np.deg2rad(np.geomspace(0.001, 2.0, 12)))
    for bb in (None, b):
        full = oracle.count_pairs(a, bb, bn, prune=False)
        win = oracle.count_pairs(a, bb, bn, prune=True)
        np.testing.assert_array_equal(full, win)
        assert full.sum() > 0


def test_rejects_bad_arguments():
    a = catalogs.uniform_box(10, 10.0, seed=1)
    with pytest.raises(ValueError):   # r_max must stay below L/2 in a periodic box
        oracle.count_pairs(a, None, Binning(MONO, [0, 5, 6], periodic=True, L=10.0))
    with pytest.raises(ValueError):   # sigma-pi needs the midpoint line of sight
        oracle.count_pairs(a, None, Binning(SIGMAPI, [0, 1], [0, 1], los=LOS_Z))


@pytest.mark.parametrize("L,rmax", [(100.0, 30.0), (100.0, 20.0), (100.0, 12.0), (100.0, 45.0)])
def test_band_prune_periodic_bands_equal_brute_force(L, rmax):
    """Periodic boxes cut into 3, 4, 8 or (below three) one band of y: the
    pruned loop equals the brute-force loop, auto and cross, including pairs
    across the faces of the box."""
    a = catalogs.mixed_periodic(1500, L, seed=61)
    b = catalogs.uniform_box(1200, L, seed=62)
    bn = Binning(MONO, np.linspace(0, rmax, 11), periodic=True, L=L)
    bm = Binning(RMU, np.linspace(0, rmax, 6), np.linspace(0, 1, 5), los=LOS_Z, periodic=True, L=L)
    for binning in (bn, bm):
        for bb in (None, b):
            full = oracle.count_pairs(a, bb, binning, prune=False)
            win = oracle.count_pairs(a, bb, binning, prune=True)
            np.testing.assert_array_equal(full, win)
            assert full.sum() > 0


@pytest.mark.parametrize("rmax", [3.0, 12.0, 60.0])
def test_band_prune_many_bands_equal_brute_force(rmax):
    """Open boxes with many bands of y (60, 17 and 4 bands over the catalog)
    and a light-cone sigma-pi case: pruned equals brute force."""
    a, b = catalogs.clustered_box_1e6(n_centres=25, per_blob=60, n_rand=1500, box=200.0)
    bn = Binning(RMU, np.linspace(0, rmax, 7), np.linspace(0, 1, 6), los=LOS_Z)
    e = np.linspace(0, rmax, 8)
    bs = Binning(SIGMAPI, e, e, los=LOS_MID)
    for binning in (bn, bs):
        for bb in (None, b):
            full = oracle.count_pairs(a, bb, binning, prune=False)
            win = oracle.count_pairs(a, bb, binning, prune=True)
            np.testing.assert_array_equal(full, win)
            assert full.sum() > 0


@pytest.mark.parametrize("periodic", [True, False])
def test_jackknife_equals_counts_of_subcatalogs(periodic):
    """Each leave-one-region-out row equals the plain brute-force count of
    the catalog without that region; the total equals the whole catalog's."""
    L = 100.0
    if periodic:
        cat = catalogs.mixed_periodic(1400, L, seed=71)
        bins = [Binning(MONO, np.linspace(0, 25, 9), periodic=True, L=L),
                Binning(RMU, np.linspace(0, 30, 7), np.linspace(0, 1, 6), los=LOS_Z,
                        periodic=True, L=L)]
        # 3 x 3 columns in (x, y) plus one region of scattered points
        reg = (np.minimum((cat.y * 3 / L).astype(int), 2) * 3
               + np.minimum((cat.x * 3 / L).astype(int), 2)).astype(np.int32)
        reg[::97] = 9
        K = 10
    else:
        cat, _ = catalogs.clustered_box_1e6(n_centres=20, per_blob=60, n_rand=10, box=150.0)
        bins = [Binning(MONO, np.linspace(0, 20, 9)),
                Binning(SIGMAPI, np.linspace(0, 15, 6), np.linspace(0, 15, 6), los=LOS_MID)]
        reg = (np.arange(len(cat)) % 5).astype(np.int32)
        K = 6   # region 5 is empty: its row equals the total
    for bn in bins:
        total, jack = oracle.count_jackknife(cat, reg, K, bn)
        np.testing.assert_array_equal(total, oracle.count_pairs(cat, None, bn))
        for k in range(K):
            sub = cat.subset(np.nonzero(reg != k)[0])
            np.testing.assert_array_equal(jack[k], oracle.count_pairs(sub, None, bn),
                                          err_msg="region %d" % k)
