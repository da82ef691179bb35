"""CPU check of the rounding analysis behind the FP32 path of the midpoint
line of sight (sigma, pi and mu of Sec. 2.1 against l = p + q).

The library's host code builds the FP32 decision thresholds of a count
(cute_fp32_decision_tables, no device work). Here the kernel's FP32
arithmetic is replayed exactly: every FP32 multiply, add and subtract is an
IEEE binary32 operation (numpy), every fused multiply-add is rounded once
from the exact rational value, and the one approximate operation the
decisions use, the hardware 1/sqrt, is replayed correctly rounded and
perturbed by 2^-22 either way (the analysis assumes at most 2^-21). On
adversarial pairs at light-cone distances (|p| around 1500 Mpc/h, separations
placed within a few rounding bands of sigma, pi and mu edges) the test checks:

* the error model: the FP32 components of s = p - q and l = p + q lie within
  the bounds ec and el from the exact rational values;
* every decision the FP32 path certifies (inside one bin, or out of range)
  agrees with the oracle's canonical FP64 classifier and with the exact
  rational sigma^2, pi^2 and mu^2;
* the bound itself: the FP32 value of sigma^2 (pi^2) differs from the exact
  rational one by no more than the band at the nearest edge plus the
  per-pair term, so every derived term is accounted for;
* the bands are not vacuous: most pairs a few bands away from an edge are
  decided in FP32.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_1210_1833_amd as cute

F32 = np.float32
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def rnd32(x: Fraction) -> float:
    """Round an exact rational to the nearest binary32 (ties to even)."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)
    scale = Fraction(2) ** (e - 23)
    q = a / scale
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return float(sign * n * scale)


def fma32(a, b, c):
    return F32(rnd32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))))


def rsq32(x, pert):
    return F32(float(np.float64(1.0) / np.sqrt(np.float64(x))) * (1.0 + pert))


class Frame:
    """The FP32 frame of one grid (autocorrelation): origin c (float64) and
    the error model of the library's planning for two such grids."""

    def __init__(self, pts, r_max):
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        self.c = 0.5 * (lo + hi)
        ext = float(np.max(0.5 * (hi - lo))) * (1.0 + 1e-12)
        rawmax = float(np.max(np.abs(pts)))
        lmax = float(np.max(np.linalg.norm(pts, axis=1))) * (1.0 + 1e-12)
        ca = float(np.max(np.abs(self.c)))
        re_ = r_max * 1.01
        # the error model a count of the grid with itself plans
        self.ec = 1.0001 * (U32 * ext + U32 * ext + U32 * re_)
        self.ec64 = 2.0 * U64 * (2 * rawmax) * 1.0001
        self.el = 1.0001 * U32 * (ext + ext + 2 * ca + (ext + 2 * ca) + 2 * lmax)
        self.el64 = 2.0 * U64 * 2 * lmax
        self.lc = F32(2.0 * self.c)

    def fp32_pair(self, p, q):
        """(s32, l32) as the kernel forms them for home p and neighbour q."""
        hp = (p - self.c).astype(np.float32)
        hq = (q - self.c).astype(np.float32)
        s = hp - hq
        ql = hq + self.lc
        l = hp + ql
        return s, l


def exact(p, q):
    P = [Fraction(float(v)) for v in p]
    Q = [Fraction(float(v)) for v in q]
    s = [a - b for a, b in zip(P, Q)]
    l = [a + b for a, b in zip(P, Q)]
    ss = sum(v * v for v in s)
    ll = sum(v * v for v in l)
    sl = sum(a * b for a, b in zip(s, l))
    return s, l, ss, ll, sl


def lightcone_points(rng, n):
    ra = rng.uniform(0.0, np.pi / 3, n)
    dec = np.arcsin(rng.uniform(0.0, 0.5, n))
    chi = rng.uniform(900.0, 2500.0, n)
    return np.stack([chi * np.cos(dec) * np.cos(ra), chi * np.cos(dec) * np.sin(ra),
                     chi * np.sin(dec)], axis=1)


def near_edge_pairs(rng, mids, edges_s, edges_p, rel):
    """Pairs (p, q) around midpoints with sigma and pi placed at edges times
    (1 + rel), rel drawn from +-[0, rel], or uniform."""
    out = []
    for m in mids:
        n = m / np.linalg.norm(m)
        e = np.cross(n, rng.normal(size=3))
        e /= np.linalg.norm(e)
        pick = rng.integers(3)
        sg = edges_s[rng.integers(1, len(edges_s))] * (1 + rng.uniform(-rel, rel))
        pi = edges_p[rng.integers(1, len(edges_p))] * (1 + rng.uniform(-rel, rel))
        if pick == 1:
            sg = rng.uniform(0.0, edges_s[-1] * 1.02)
        elif pick == 2:
            pi = rng.uniform(0.0, edges_p[-1] * 1.02)
        s = sg * e + pi * n
        out.append((m + 0.5 * s, m - 0.5 * s))
    return out


def sp_decisions(fr, b1, b2, k, p, q, pert):
    """The FP32 sigma-pi path of the kernel: ('in', k1, k2), 'out' or None
    (re-tested), for every bin (the kernel tests the estimated one)."""
    s, l = fr.fp32_pair(p, q)
    dx, dy, dz = s
    lx, ly, lz = l
    v = fma32(dz, dz, fma32(dy, dy, dx * dx))
    sl = fma32(dz, lz, fma32(dy, ly, dx * lx))
    ll = fma32(lz, lz, fma32(ly, ly, lx * lx))
    sl2 = sl * sl
    c2 = fma32(v, ll, -sl2)
    rl = rsq32(ll, pert)
    t = fma32(F32(k["K1"]), ll * rl, F32(k["K0"]))
    vin = v < F32(k["skip32"])
    lg = ll >= F32(k["llg"])
    # a bin's entry (m, H): inside when |F + m ll| <= H ll - t
    nt = -t
    ins = [abs(float(fma32(F32(b1[i, 0]), ll, c2))) <= float(fma32(F32(b1[i, 1]), ll, nt))
           for i in range(len(b1))]
    inp = [abs(float(fma32(F32(b2[j, 0]), ll, sl2))) <= float(fma32(F32(b2[j, 1]), ll, nt))
           for j in range(len(b2))]
    top = (fma32(F32(k["w_sigma_top"]), ll, c2) >= t) or (fma32(F32(k["w_pi_top"]), ll, sl2) >= t)
    if k["low"]:
        top = top or (fma32(F32(k["w_sigma_bottom"]), ll, c2) <= -t) or \
            (fma32(F32(k["w_pi_bottom"]), ll, sl2) <= -t)
    certified = [(i, j) for i in range(len(b1)) for j in range(len(b2))
                 if vin and lg and ins[i] and inp[j]]
    out = (not vin) or (lg and top)
    return certified, out, dict(v=v, ll=ll, c2=c2, sl2=sl2, t=t, s=s, l=l)


@pytest.mark.parametrize("first", [0.0, 3.0])
def test_sigma_pi_bands_on_adversarial_light_cone_pairs(first):
    rng = np.random.default_rng(20240 + int(first))
    es_ = np.linspace(first, 150.0, 76 if first == 0.0 else 74)
    ep_ = np.linspace(first, 150.0, 76 if first == 0.0 else 74)
    bn = cute.Binning(cute.BIN_SIGMAPI, es_, ep_, los=cute.LOS_MIDPOINT)
    ob = oracle.Binning(oracle.SIGMAPI, es_, ep_, los=oracle.LOS_MID)
    r_max = math.hypot(150.0, 150.0) * (1 + 1e-12)
    mids = lightcone_points(rng, 900)
    pairs = near_edge_pairs(rng, mids, es_, ep_, 3e-6) + near_edge_pairs(rng, mids[:300], es_, ep_, 1e-3)
    allp = np.array([x for pq in pairs for x in pq])
    fr = Frame(allp, r_max)
    b1, b2, k = cute.fp32_decision_tables(bn, fr.ec, fr.ec64, fr.el, fr.el64)
    S2 = [Fraction(float(e * e)) for e in es_]
    P2 = [Fraction(float(e * e)) for e in ep_]
    n2 = len(ep_) - 1
    decided = far = far_decided = 0
    worst = 0.0
    for idx, (p, q) in enumerate(pairs):
        s_ex, l_ex, ss, lle, sle = exact(p, q)
        sig2 = (ss * lle - sle * sle) / lle
        pi2 = sle * sle / lle
        canon = oracle.classify(p, q, ob)
        for pert in (-2.0 ** -22, 0.0, 2.0 ** -22):
            cert, out, w = sp_decisions(fr, b1, b2, k, p, q, pert)
            # error model
            assert max(abs(Fraction(float(a)) - b) for a, b in zip(w["s"], s_ex)) <= fr.ec
            assert max(abs(Fraction(float(a)) - b) for a, b in zip(w["l"], l_ex)) <= fr.el
            assert len(cert) <= 1
            if cert:
                i, j = cert[0]
                assert canon == i * n2 + j, (idx, cert, canon, float(sig2), float(pi2))
                assert S2[i] <= sig2 < S2[i + 1] and P2[j] <= pi2 < P2[j + 1]
            if out:
                assert canon == -1, (idx, canon, float(sig2), float(pi2))
                assert not cert
            if pert == 0.0:
                decided += bool(cert) or out
                # margin of the pair from its nearest edges, in bands
                ks = min(range(len(S2)), key=lambda a: abs(S2[a] - sig2))
                kp = min(range(len(P2)), key=lambda a: abs(P2[a] - pi2))
                ll = float(w["ll"])
                # the certified interval of bin j is about [-m - H, -m + H]; the
                # band at an edge is its distance from the edge
                def upper(b, j):
                    return -float(b[j, 0]) + float(b[j, 1])

                def lower(b, j):
                    return -float(b[j, 0]) - float(b[j, 1])
                bs_lo = lower(b1, min(ks, len(b1) - 1)) - float(S2[ks]) if S2[ks] > 0 else 0.0
                # the bound: |FP32 sigma^2 - exact| <= band + t / ll
                band_s = abs(upper(b1, ks - 1) - float(S2[ks])) if ks > 0 else bs_lo
                band_p = abs(upper(b2, kp - 1) - float(P2[kp])) if kp > 0 else 0.0
                tl = float(w["t"]) / ll
                sig2_32 = float(w["c2"]) / ll
                pi2_32 = float(w["sl2"]) / ll
                if float(ss) < r_max ** 2:
                    if ks > 0:
                        worst = max(worst, abs(sig2_32 - float(sig2)) / (band_s + tl))
                    if kp > 0:
                        worst = max(worst, abs(pi2_32 - float(pi2)) / (band_p + tl))
                    margin = min(abs(float(sig2 - S2[ks])) / max(band_s + tl, 1e-300),
                                 abs(float(pi2 - P2[kp])) / max(band_p + tl, 1e-300))
                    if margin > 4.0:
                        far += 1
                        far_decided += bool(cert) or out
    # the FP32 evaluation error stays inside the derived band
    assert worst <= 1.0, worst
    # pairs more than four bands from every edge are decided in FP32
    assert far > 100 and far_decided == far, (far, far_decided)
    # most pairs sit within a few bands of an edge by construction; still a
    # good share is decided in FP32
    assert decided > 0.15 * len(pairs)


def test_mu_midpoint_bands_on_adversarial_light_cone_pairs():
    rng = np.random.default_rng(31337)
    re_ = np.arange(41) * 5.0
    me = np.arange(51) / 50.0
    bn = cute.Binning(cute.BIN_RMU, re_, me, los=cute.LOS_MIDPOINT)
    ob = oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_MID)
    mids = lightcone_points(rng, 1500)
    pairs = []
    for m in mids:
        n = m / np.linalg.norm(m)
        e = np.cross(n, rng.normal(size=3))
        e /= np.linalg.norm(e)
        near = len(pairs) % 2 == 0
        mu = me[rng.integers(0, 51)] * (1 + rng.uniform(-1e-5, 1e-5)) if near else rng.uniform()
        mu = min(mu, 1.0)
        r = rng.uniform(0.5, 199.0) if rng.integers(2) else re_[rng.integers(1, 41)] * (1 + 1e-7)
        s = r * (mu * n + math.sqrt(max(0.0, 1 - mu * mu)) * e)
        pairs.append((m + 0.5 * s, m - 0.5 * s))
    allp = np.array([x for pq in pairs for x in pq])
    fr = Frame(allp, 200.0)
    b1_unused, b2_unused, k = cute.fp32_decision_tables(bn, fr.ec, fr.ec64, fr.el, fr.el64)
    M2 = [Fraction(float(x * x)) for x in me]
    n2 = 50
    decided = 0   # pairs with a uniform mu (odd index) decided in FP32
    for idx, (p, q) in enumerate(pairs):
        _, _, ss, lle, sle = exact(p, q)
        canon = oracle.classify(p, q, ob)
        for pert in (-2.0 ** -22, 0.0, 2.0 ** -22):
            s, l = fr.fp32_pair(p, q)
            dx, dy, dz = s
            lx, ly, lz = l
            v = fma32(dz, dz, fma32(dy, dy, dx * dx))
            sl = fma32(dz, lz, fma32(dy, ly, dx * lx))
            ll = fma32(lz, lz, fma32(ly, ly, lx * lx))
            r = v * rsq32(v, pert)
            w = v * ll
            sl2 = sl * sl
            lnorm = ll * rsq32(ll, pert)
            c = {n_: F32(k[n_]) for n_ in ("A0", "A1", "A2", "B0", "B1", "B2", "C2", "C0")}
            delta = fma32(ll, fma32(c["A2"], v, fma32(c["A1"], r, c["A0"])),
                          fma32(lnorm, fma32(c["B2"], v, fma32(c["B1"], r, c["B0"])),
                                fma32(c["C2"], v, c["C0"])))
            lg = ll >= F32(k["llg"])
            for j in range(n2):
                lo = F32(-M2[j]) if M2[j] > 0 else F32(1e30)
                hi = F32(-M2[j + 1]) if j + 1 < n2 else F32(-1e30)
                flo = fma32(lo, w, sl2)
                fhi = fma32(hi, w, sl2)
                if lg and flo >= delta and fhi <= -delta:
                    # mu certified in bin j: the canonical and exact mu bins agree
                    if canon >= 0:
                        assert canon % n2 == j, (idx, j, canon)
                    mu2 = sle * sle / (ss * lle)
                    assert M2[j] <= mu2 and (mu2 < M2[j + 1] or j == n2 - 1)
                    if pert == 0.0 and idx % 2 == 1:
                        decided += 1
    # pairs at a uniform mu are almost always decided in FP32
    assert decided > 0.9 * (len(pairs) // 2), decided
