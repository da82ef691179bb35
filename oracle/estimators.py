"""Exact-arithmetic 2PCF estimators and multipoles (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every estimator below is evaluated in exact rational arithmetic
(``fractions.Fraction``) on the integer pair counts, then rounded to the
nearest double once.

* Natural estimator (Sec. 2.2): xi_N = N_r(N_r-1)/(N_d(N_d-1)) * DD/RR - 1.
* Landy-Szalay (Sec. 2.2): xi_LS = [N_r(N_r-1)/(N_d(N_d-1)) DD
  - (N_r-1)/N_d DR + RR] / RR, with DD and RR counting unordered pairs and DR
  all data-random pairs.
* Periodic box (Sec. 2.2, the estimator for a catalog without boundaries):
  1 + xi = (pair count) / (expected count of a uniform catalog). Reading taken
  here: with unordered pairs the expected count in the shell [e_k, e_{k+1}) is
  N(N-1)/2 * V_k / L^3 with the exact shell volume V_k = 4/3 pi
  (e_{k+1}^3 - e_k^3), instead of the paper's N^2 v(r)/V with v = 4 pi r^2 dr.
  pi enters through a 60-digit rational approximation, so the result is
  exact to far below double precision.
* Multipoles (Sec. 2.1, the Legendre expansion of xi(r, mu) and the monopole
  as the average over mu): with mu = |cos| in [0, 1] and xi even in mu,
  xi_l(r) = (2l+1) int_0^1 xi(r, mu) P_l(mu) dmu for even l; xi is taken
  constant within each mu bin and the integral of P_l over each bin is done
  exactly on the rational Legendre polynomial.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

PI_60 = Fraction("3.141592653589793238462643383279502884197169399375105820974944")


def _q(v) -> Fraction:
    """Exact rational value of an integer or a binary64 number."""
    if isinstance(v, (int, np.integer)):
        return Fraction(int(v))
    return Fraction(float(v))


def _to_float(f: Fraction) -> float:
    return float(f)  # Fraction -> float is correctly rounded


def natural(dd, rr, nd: int, nr: int):
    dd = np.asarray(dd)
    rr = np.asarray(rr)
    out = np.empty(dd.shape, dtype=np.float64)
    a = Fraction(nr * (nr - 1), nd * (nd - 1))
    for idx in np.ndindex(dd.shape):
        r = int(rr[idx])
        if r == 0:
            out[idx] = np.nan
            continue
        out[idx] = _to_float(a * int(dd[idx]) / r - 1)
    return out


def landy_szalay(dd, dr, rr, nd: int, nr: int):
    dd, dr, rr = np.asarray(dd), np.asarray(dr), np.asarray(rr)
    out = np.empty(dd.shape, dtype=np.float64)
    a = Fraction(nr * (nr - 1), nd * (nd - 1))
    b = Fraction(nr - 1, nd)
    for idx in np.ndindex(dd.shape):
        r = int(rr[idx])
        if r == 0:
            out[idx] = np.nan
            continue
        out[idx] = _to_float((a * int(dd[idx]) - b * int(dr[idx]) + r) / r)
    return out


def shell_volume(e_lo, e_hi) -> Fraction:
    lo, hi = _q(e_lo), _q(e_hi)
    return Fraction(4, 3) * PI_60 * (hi ** 3 - lo ** 3)


def box(dd, nd: int, box_size: float, edges):
    """Periodic-box estimator for a MONO histogram (unordered pairs)."""
    dd = np.asarray(dd)
    edges = np.asarray(edges, dtype=np.float64)
    vol = _q(box_size) ** 3
    npairs = Fraction(nd * (nd - 1), 2)
    out = np.empty(dd.shape, dtype=np.float64)
    for k in range(dd.shape[0]):
        expect = npairs * shell_volume(edges[k], edges[k + 1]) / vol
        if expect == 0:
            out[k] = np.nan
            continue
        out[k] = _to_float(Fraction(int(dd[k])) / expect - 1)
    return out


# ---------------------------------------------------------------------------
# Legendre polynomials as exact rational coefficient lists (lowest order first)
# ---------------------------------------------------------------------------
def legendre_poly(ell: int):
    """Coefficients of P_ell from Bonnet's recursion
    (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}."""
    p_prev = [Fraction(1)]
    if ell == 0:
        return p_prev
    p = [Fraction(0), Fraction(1)]
    for n in range(1, ell):
        xp = [Fraction(0)] + p
        nxt = []
        for i in range(n + 2):
            a = xp[i] * (2 * n + 1) if i < len(xp) else Fraction(0)
            b = p_prev[i] * n if i < len(p_prev) else Fraction(0)
            nxt.append((a - b) / (n + 1))
        p_prev, p = p, nxt
    return p


def _antideriv_at(coeffs, x: Fraction) -> Fraction:
    return sum(c * x ** (i + 1) / (i + 1) for i, c in enumerate(coeffs))


def multipoles(xi_rmu, mu_edges, ells):
    """xi_l(r_i) for even l from a piecewise-constant xi(r_i, mu) table."""
    xi = np.asarray(xi_rmu, dtype=np.float64)
    mu = [_q(m) for m in np.asarray(mu_edges, dtype=np.float64)]
    out = np.empty((len(ells), xi.shape[0]), dtype=np.float64)
    for a, ell in enumerate(ells):
        if ell < 0 or ell % 2:
            raise ValueError("multipoles are defined here for even l >= 0")
        c = legendre_poly(ell)
        w = [(2 * ell + 1) * (_antideriv_at(c, mu[j + 1]) - _antideriv_at(c, mu[j]))
             for j in range(len(mu) - 1)]
        for i in range(xi.shape[0]):
            s = Fraction(0)
            for j in range(len(w)):
                s += Fraction(float(xi[i, j])) * w[j]
            out[a, i] = _to_float(s)
    return out


def multipole_weights_abs(mu_edges, ell):
    """|(2l+1) int_bin P_l| per mu bin, used for the tolerance scale."""
    mu = [_q(m) for m in np.asarray(mu_edges, dtype=np.float64)]
    c = legendre_poly(ell)
    return np.array([float(abs((2 * ell + 1) * (_antideriv_at(c, mu[j + 1])
                                                - _antideriv_at(c, mu[j]))))
                     for j in range(len(mu) - 1)])
