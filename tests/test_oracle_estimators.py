"""Pins of the oracle's estimators (Sec. 2.2) and multipoles (Sec. 2.1)."""
import json
import math
import os

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy import integrate, special

import catalogs
import oracle
from oracle import MONO, Binning
from oracle import estimators as est

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_hand_worked_estimators():
    with open(os.path.join(GOLDEN, "estimator_example.json")) as f:
        g = json.load(f)
    nat = est.natural(g["dd"], g["rr"], g["nd"], g["nr"])
    ls = est.landy_szalay(g["dd"], g["dr"], g["rr"], g["nd"], g["nr"])
    for got, want in ((nat, g["natural"]), (ls, g["landy_szalay"])):
        for a, b in zip(got, want):
            if b is None:
                assert math.isnan(a)
            else:
                assert a == b


def test_proportional_counts_give_zero():
    """DD, DR, RR in the ratios of the pair totals -> xi_N = xi_LS = 0 exactly."""
    nd, nr = 1000, 3000
    c = np.array([1, 7, 123456, 2])
    dd = c * nd * (nd - 1)          # proportional to N_d(N_d-1)/2
    dr = c * 2 * nd * nr            # proportional to N_d N_r
    rr = c * nr * (nr - 1)          # proportional to N_r(N_r-1)/2
    assert np.all(est.natural(dd, rr, nd, nr) == 0.0)
    assert np.all(est.landy_szalay(dd, dr, rr, nd, nr) == 0.0)


def test_box_estimator_is_unbiased_for_uniform_points():
    cat = catalogs.periodic_uniform_2e4()
    edges = np.arange(31) * 5.0
    dd = oracle.count_pairs(cat, None, Binning(MONO, edges, periodic=True, L=1000.0), prune=True)
    xi = est.box(dd, len(cat), 1000.0, edges)
    n = len(cat)
    p = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3) / 1000.0 ** 3
    mean = n * (n - 1) / 2 * p
    sd_xi = np.sqrt(mean * (1 - p)) / mean
    assert np.all(np.abs(xi) < 5 * sd_xi)
    # an exactly expected count gives xi = 0 up to the rounding of the count
    exp = np.rint(mean).astype(np.int64)
    xi0 = est.box(exp, n, 1000.0, edges)
    assert np.all(np.abs(xi0) <= 0.5 / mean + 1e-15)


def test_legendre_coefficients_match_numpy():
    for ell in range(0, 9):
        mine = [float(c) for c in est.legendre_poly(ell)]
        ref = npleg.leg2poly([0] * ell + [1])
        np.testing.assert_allclose(mine, ref, rtol=1e-13, atol=1e-15)


def test_multipoles_closed_forms():
    mu = np.linspace(0, 1, 51)
    xi = np.full((4, 50), 0.37)
    m = est.multipoles(xi, mu, [0, 2, 4])
    np.testing.assert_allclose(m[0], 0.37, rtol=1e-15)
    assert np.all(np.abs(m[1]) <= 1e-15) and np.all(np.abs(m[2]) <= 1e-15)


def test_multipoles_match_numerical_quadrature():
    """Independent route: quadrature of the piecewise-constant xi(mu) P_l(mu)."""
    g = np.random.Generator(np.random.PCG64(3))
    mu = np.sort(np.concatenate([[0.0, 1.0], g.random(9)]))
    xi = g.normal(size=(3, len(mu) - 1))
    ells = [0, 2, 4, 6]
    m = est.multipoles(xi, mu, ells)
    for a, ell in enumerate(ells):
        for i in range(xi.shape[0]):
            tot = 0.0
            for j in range(len(mu) - 1):
                v, _ = integrate.quad(lambda t: special.eval_legendre(ell, t), mu[j], mu[j + 1],
                                      epsabs=1e-15, epsrel=1e-14)
                tot += xi[i, j] * v
            assert abs(m[a, i] - (2 * ell + 1) * tot) < 1e-12
    # xi(mu) = P_2 exactly recovers xi_2 = 1 in the limit of fine bins
    fine = np.linspace(0, 1, 2001)
    mids = 0.5 * (fine[1:] + fine[:-1])
    m2 = est.multipoles(special.eval_legendre(2, mids)[None, :], fine, [0, 2, 4])
    assert abs(m2[0, 0]) < 1e-6 and abs(m2[1, 0] - 1) < 1e-6 and abs(m2[2, 0]) < 1e-6
