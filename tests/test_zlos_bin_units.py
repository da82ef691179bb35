"""CPU check of the rounding analysis behind the FP32 path of the z line of
sight, where r and mu (Sec. 2.1: mu = |dz| / r) are decided in bin units.

The library's host code builds the constants of a count
(cute_fp32_zlos_constants, no device work). Here the kernel's FP32
arithmetic is replayed exactly: every FP32 multiply and subtract is an IEEE
binary32 operation (numpy), every fused multiply-add is rounded once from the
exact rational value, and the hardware 1/sqrt is replayed correctly rounded
and perturbed by 2^-21 either way (the most the analysis allows). The
kernel forms, for a pair with FP32 separation s:

    v = |s|^2, ts = fl(v rsq(v) + s1), k = round(ts e1a) clamped to the bins,
    certified in r bin k when |fl(ts e1a - k)| <= rB0;
    ts2 = fl(|s_z| rsq(v) + s2), j likewise, certified in mu bin j when
    |fl(ts2 e2a - j)| <= fl(muB1 rsq(v) + muB0);
    out of range when v >= out_hi.

On adversarial pairs (separations within a few rounding bands of r and mu
edges, at the coordinates of the benchmark's open box and far from the
origin) the test checks:

* the error model: the FP32 components of s lie within ec of the exact ones;
* every pair the FP32 path certifies (inside one bin, or out of range) agrees
  with the oracle's canonical FP64 classifier and with the exact rational
  r^2 and mu^2;
* the bound: the FP32 positions in bin units differ from the exact ones
  (a (r + s1), a (mu + s2)) by less than the half-width removed from the bin
  (1/2 - rB0, and 1/2 - muB0 - muB1 / r);
* the bands are not vacuous: pairs far from every edge are decided in FP32.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_1210_1833_amd as cute
from test_midpoint_bands import F32, U32, U64, fma32, rsq32

getcontext().prec = 50
TWO23 = F32(2.0 ** 23)


def frame_of(pts, r_max):
    """FP32 frame (centre) and error model of a grid counted with itself."""
    lo, hi = pts.min(axis=0), pts.max(axis=0)
    c = 0.5 * (lo + hi)
    ext = float(np.max(0.5 * (hi - lo))) * (1.0 + 1e-12)
    rawmax = float(np.max(np.abs(pts)))
    ec = 1.0001 * (U32 * ext + U32 * ext + U32 * r_max * 1.01)
    ec64 = 2.0 * U64 * (2 * rawmax) * 1.0001
    return c, ec, ec64


def est(ts, a, n):
    """The kernel's clamped bin estimate and the offset from its centre."""
    e = fma32(ts, a, TWO23)
    # the clamp is on the float's bits, monotone for positive floats; floats
    # in [2^23, 2^24) are integers, the one below 2^23 clamps to bin 0
    k = min(max(float(e) - 2.0 ** 23, 0.0), float(n - 1))
    off = fma32(ts, a, TWO23 - F32(2.0 ** 23 + k))
    return int(k), off


def replay(k, c, p, q, n1, n2, pert):
    hp = (p - c).astype(np.float32)
    hq = (q - c).astype(np.float32)
    dx, dy, dz = hp - hq
    v = fma32(dz, dz, fma32(dy, dy, dx * dx))
    rinv = rsq32(v, pert)
    ts = fma32(v, rinv, F32(k["s1"]))
    kb, offr = est(ts, F32(k["e1a"]), n1)
    ts2 = fma32(abs(dz), rinv, F32(k["s2"]))
    kmb, offm = est(ts2, F32(k["e2a"]), n2)
    half = fma32(F32(k["muB1"]), rinv, F32(k["muB0"]))
    rin = abs(float(offr)) <= float(F32(k["rB0"]))
    mbin = abs(float(offm)) <= float(half)
    out = float(v) >= float(F32(k["out_hi"]))
    return dict(s=(dx, dy, dz), v=v, ts=ts, ts2=ts2, kb=kb, kmb=kmb, half=half,
                cert=rin and mbin, out=out)


def make_pairs(rng, n, re_, me, box, offset):
    mids = rng.uniform(0.0, box, (n, 3)) + offset
    pairs = []
    for i, m in enumerate(mids):
        kind = i % 6
        tight = rng.integers(2) == 1   # half of the near-edge pairs much closer
        dr, dm = (2e-8, 3e-8) if tight else (2e-6, 3e-6)
        if kind == 0:     # near an r edge
            r = re_[rng.integers(1, len(re_))] * (1 + rng.uniform(-dr, dr))
            mu = rng.uniform()
        elif kind == 1:   # near a mu edge
            r = rng.uniform(0.5, re_[-1] * 1.02)
            mu = me[rng.integers(0, len(me))] * (1 + rng.uniform(-dm, dm))
        elif kind == 2:   # near both
            r = re_[rng.integers(1, len(re_))] * (1 + rng.uniform(-dr, dr))
            mu = me[rng.integers(0, len(me))] * (1 + rng.uniform(-dm, dm))
        elif kind == 3:   # tiny separations and the top edge
            r = rng.choice([rng.uniform(1e-4, 1e-2), re_[-1] * (1 + rng.uniform(-1e-5, 1e-5))])
            mu = rng.uniform()
        else:             # anywhere, some past r_max
            r = rng.uniform(0.0, re_[-1] * 1.1)
            mu = rng.uniform()
        mu = min(max(mu, 0.0), 1.0)
        ph = rng.uniform(0.0, 2 * np.pi)
        sxy = r * math.sqrt(max(0.0, 1 - mu * mu))
        s = np.array([sxy * math.cos(ph), sxy * math.sin(ph), r * mu * (1 if rng.integers(2) else -1)])
        pairs.append((m + 0.5 * s, m - 0.5 * s))
    return pairs


@pytest.mark.parametrize("case", ["bench", "far"])
def test_zlos_bin_unit_decisions_on_adversarial_pairs(case):
    rng = np.random.default_rng(4242 if case == "bench" else 4343)
    if case == "bench":
        re_, me, box, offset = np.arange(41) * 5.0, np.arange(51) / 50.0, 2000.0, 0.0
    else:
        re_, me, box, offset = np.arange(31) * 5.0, np.arange(26) / 25.0, 3000.0, 2.0e4
    n1, n2 = len(re_) - 1, len(me) - 1
    bn = cute.Binning(cute.BIN_RMU, re_, me, los=cute.LOS_Z)
    ob = oracle.Binning(oracle.RMU, re_, me, los=oracle.LOS_Z)
    pairs = make_pairs(rng, 2400, re_, me, box, offset)
    allp = np.array([x for pq in pairs for x in pq])
    c, ec, ec64 = frame_of(allp, re_[-1])
    k = cute.fp32_zlos_constants(bn, ec, ec64)
    assert k["path"] == 2.0, k   # r and mu both in bin units
    assert 0.0 < k["rB0"] < 0.5 and k["muB1"] <= 0.0 < k["muB0"] < 0.5
    R2 = [Fraction(float(e * e)) for e in re_]
    M2 = [Fraction(float(e * e)) for e in me]
    e1a, s1, e2a, s2 = (Fraction(float(F32(k[n]))) for n in ("e1a", "s1", "e2a", "s2"))
    decided = far = far_decided = 0
    worst_r = worst_m = 0.0
    for idx, (p, q) in enumerate(pairs):
        P = [Fraction(float(x)) for x in p]
        Q = [Fraction(float(x)) for x in q]
        s_ex = [a - b for a, b in zip(P, Q)]
        r2 = sum(x * x for x in s_ex)
        canon = oracle.classify(p, q, ob)
        r_ex = Fraction((Decimal(r2.numerator) / Decimal(r2.denominator)).sqrt())
        mu2 = s_ex[2] * s_ex[2] / r2 if r2 > 0 else Fraction(0)
        mu_ex = abs(s_ex[2]) / r_ex if r2 > 0 else Fraction(0)
        for pert in (-2.0 ** -21, 0.0, 2.0 ** -21):
            w = replay(k, c, p, q, n1, n2, pert)
            assert max(abs(Fraction(float(a)) - b) for a, b in zip(w["s"], s_ex)) <= ec
            if w["cert"]:
                assert canon == w["kb"] * n2 + w["kmb"], (idx, canon, w["kb"], w["kmb"], float(r2), float(mu2))
                assert R2[w["kb"]] <= r2 < R2[w["kb"] + 1]
                assert M2[w["kmb"]] <= mu2 and (mu2 < M2[w["kmb"] + 1] or w["kmb"] == n2 - 1)
            if w["out"]:
                assert canon == -1, (idx, canon, float(r2))
            if pert == 0.0 and r2 > 0:
                # the positions in bin units against the exact ones
                x1 = Fraction(float(w["ts"])) * e1a
                x1_ex = e1a * (r_ex + s1)
                x2 = Fraction(float(w["ts2"])) * e2a
                x2_ex = e2a * (mu_ex + s2)
                if r2 < R2[-1]:
                    worst_r = max(worst_r, float(abs(x1 - x1_ex)) / (0.5 - k["rB0"]))
                    worst_m = max(worst_m, float(abs(x2 - x2_ex)) / (0.5 - float(w["half"])))
                decided += bool(w["cert"]) or w["out"]
                # margin from the nearest edges in bin units, in bands
                fr = float(abs(x1_ex - round(x1_ex))), float(abs(x2_ex - round(x2_ex)))
                if r2 < R2[-1] * Fraction(99, 100) and min(0.5 - fr[0], 0.5 - fr[1]) > 4 * max(
                        0.5 - k["rB0"], 0.5 - float(w["half"])) and mu_ex < 1:
                    far += 1
                    far_decided += bool(w["cert"])
    assert worst_r <= 1.0 and worst_m <= 1.0, (worst_r, worst_m)
    assert far > 200 and far_decided == far, (far, far_decided)
    assert decided > 0.3 * len(pairs)


def test_zlos_constants_paths():
    """Which bin-unit path a z line-of-sight count takes."""
    me = np.arange(51) / 50.0
    lin = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, me, los=cute.LOS_Z)
    assert cute.fp32_zlos_constants(lin, 1e-4, 1e-12)["path"] == 2.0
    logr = cute.Binning(cute.BIN_RMU, np.logspace(-1, 2, 31), me, los=cute.LOS_Z)
    assert cute.fp32_zlos_constants(logr, 1e-4, 1e-12)["path"] == 3.0
    # r bins starting above 0 and a partial mu range keep the band tables
    rmin = cute.Binning(cute.BIN_RMU, 1.0 + np.arange(41) * 5.0, me, los=cute.LOS_Z)
    assert cute.fp32_zlos_constants(rmin, 1e-4, 1e-12)["path"] in (0.0, 1.0)
    part = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, np.arange(26) / 50.0, los=cute.LOS_Z)
    assert cute.fp32_zlos_constants(part, 1e-4, 1e-12)["path"] in (0.0, 1.0)
    # r bins so fine against the coordinate error that the r band would be a
    # large part of a bin: the band tables again
    fine = cute.Binning(cute.BIN_RMU, np.linspace(0.0, 0.01, 21), me, los=cute.LOS_Z)
    assert cute.fp32_zlos_constants(fine, 6e-5, 1e-12)["path"] in (0.0, 1.0)
    assert cute.fp32_zlos_constants(fine, 1e-9, 1e-15)["path"] == 2.0
    mid = cute.Binning(cute.BIN_RMU, np.arange(41) * 5.0, me, los=cute.LOS_MIDPOINT)
    with pytest.raises(cute.CuteError):
        cute.fp32_zlos_constants(mid, 1e-4, 1e-12)
