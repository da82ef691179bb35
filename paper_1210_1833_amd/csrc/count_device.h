// Device code of the pair-count kernels, shared by the single-count kernel
// and the batched kernel (each translation unit instantiates what it uses).
#pragma once

#include <math.h>
#include <stdint.h>

#include "cute_internal.h"
#include "runtime.h"

namespace cute {

namespace {

constexpr uint32_t kNoBin = 0xffffffffu;
constexpr double kPi = 3.14159265358979323846264338327950288;

// Read-only device memory seen through the constant address space: loads at
// wave-uniform addresses become scalar (s_load) loads into SGPRs.
typedef const __attribute__((address_space(4))) float* cfp;
typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) uint32_t* cu32p;
typedef const __attribute__((address_space(4))) double* cf64p;

// x, y, z of the U consecutive points h .. h+U-1 from one base address with
// constant offsets (the index is widened before the offsets are added, so the
// scalar loads share one address computation and can merge)
template <uint32_t U>
__device__ __forceinline__ void load_points32(const float4* p, uint32_t h, float* x, float* y,
                                              float* z) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(4))) f4v* cf4p;
    const cf4p f = (cf4p)(const void*)(p + h);
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        const f4v q = f[u];
        x[u] = q.x;
        y[u] = q.y;
        z[u] = q.z;
    }
}
template <uint32_t U>
__device__ __forceinline__ void load_points64(const P64* p, uint32_t h, double* x, double* y,
                                              double* z) {
    const cdp f = (cdp)(const void*)(p + h);
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        x[u] = f[4 * u];
        y[u] = f[4 * u + 1];
        z[u] = f[4 * u + 2];
    }
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int unii(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }

// ---------------------------------------------------------------------------
// Canonical FP64 classification (identical predicates to a plain FP64 double
// loop: squared quantities against squared edges, explicit fused multiply-adds,
// no square root or division). dx, dy, dz are the separation p - q (minimum
// image already applied), l the sum p + q (midpoint line of sight).
// Returns the flattened bin or kNoBin.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int last_le64(const double* t, int n, double v, int k) {
    // largest k in [0, n-1] with t[k] <= v, given t[0] <= v < t[n]; k is a guess
    while (k > 0 && v < t[k]) k--;
    while (k < n - 1 && v >= t[k + 1]) k++;
    return k;
}

__device__ __forceinline__ int last_ratio64(const double* t, int n, double num, double den,
                                            int k) {
    // largest k in [0, n-1] with num >= t[k] * den, given it holds at 0
    while (k > 0 && !(num >= t[k] * den)) k--;
    while (k < n - 1 && num >= t[k + 1] * den) k++;
    return k;
}

template <int MODE>
__device__ __forceinline__ uint32_t classify64(const CountArgs& P, const double* T1,
                                               const double* T2, double dx, double dy, double dz,
                                               double lx, double ly, double lz, int k1g,
                                               int k2g) {
    const int n1 = P.n1, n2 = P.n2;
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (MODE == M_MONO || MODE == M_THETA) {
        if (!(T1[0] <= d2 && d2 < T1[n1])) return kNoBin;
        return (uint32_t)last_le64(T1, n1, d2, k1g);
    }
    if (MODE == M_RMU_Z || MODE == M_RMU_MID) {
        if (!(T1[0] <= d2 && d2 < T1[n1])) return kNoBin;
        int ir = last_le64(T1, n1, d2, k1g);
        double num, den;
        if (MODE == M_RMU_Z) {
            num = dz * dz;
            den = d2;
        } else {
            double sl = fma(dz, lz, fma(dy, ly, dx * lx));
            double ll = fma(lz, lz, fma(ly, ly, lx * lx));
            if (ll == 0.0) {
                num = 0.0;
                den = 1.0;
            } else {
                num = sl * sl;
                den = d2 * ll;
            }
        }
        if (d2 == 0.0) {
            num = 0.0;
            den = 1.0;
        }
        if (!(num >= T2[0] * den)) return kNoBin;
        if (!P.mu_top_closed && num >= T2[n2] * den) return kNoBin;
        int im = last_ratio64(T2, n2, num, den, k2g);
        return (uint32_t)(ir * n2 + im);
    }
    // SIGMAPI, midpoint line of sight
    double sl = fma(dz, lz, fma(dy, ly, dx * lx));
    double ll = fma(lz, lz, fma(ly, ly, lx * lx));
    double cx = fma(dy, lz, -(dz * ly));
    double cy = fma(dz, lx, -(dx * lz));
    double cz = fma(dx, ly, -(dy * lx));
    double c2 = fma(cz, cz, fma(cy, cy, cx * cx));
    double sn, pn, den;
    if (ll == 0.0) {
        sn = d2;
        pn = 0.0;
        den = 1.0;
    } else {
        sn = c2;
        pn = sl * sl;
        den = ll;
    }
    if (!(sn >= T1[0] * den)) return kNoBin;
    if (sn >= T1[n1] * den) return kNoBin;
    if (!(pn >= T2[0] * den)) return kNoBin;
    if (pn >= T2[n2] * den) return kNoBin;
    int is = last_ratio64(T1, n1, sn, den, k1g);
    int ip = last_ratio64(T2, n2, pn, den, k2g);
    return (uint32_t)(is * n2 + ip);
}

// Guess of the dimension-1 bin from a float value (used to start the exact
// search; any guess in range gives the right answer).
template <int MODE, int EST>
__device__ __forceinline__ int guess1(const CountArgs& P, float v) {
    float t;
    if (MODE == M_THETA) {
        float c = __builtin_amdgcn_sqrtf(v);
        float th = fmaf(c * v, 1.0f / 24.0f, c);  // 2 asin(c/2) to third order
        t = est_log(EST) ? __builtin_amdgcn_logf(th) : th;
    } else {
        t = est_log(EST) ? __builtin_amdgcn_logf(v) : __builtin_amdgcn_sqrtf(v);
    }
    return (int)__builtin_amdgcn_fmed3f(fmaf(t, P.e1a, P.e1b), 0.0f, P.n1m1);
}

// clamp to [0, n-1] with one v_med3; a NaN estimate converts to bin 0 or is
// clamped, so the index always stays in range
__device__ __forceinline__ int guess_lin(float t, float a, float b, float nm1) {
    return (int)__builtin_amdgcn_fmed3f(fmaf(t, a, b), 0.0f, nm1);
}

// Canonical classification of a queued pair from the sorted FP64 copies.
template <int MODE, int EST>
__device__ uint32_t classify_pair64(const CountArgs& P, const double* T1, const double* T2,
                                    const P64& p, const P64& q) {
    double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    if (P.periodic) {
        const double L = P.L, h = 0.5 * P.L;
        dx = dx > h ? dx - L : (dx < -h ? dx + L : dx);
        dy = dy > h ? dy - L : (dy < -h ? dy + L : dy);
        dz = dz > h ? dz - L : (dz < -h ? dz + L : dz);
    }
    double lx = p.x + q.x, ly = p.y + q.y, lz = p.z + q.z;
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    float v = (float)d2;
    int k1, k2 = 0;
    if (MODE == M_SIGMAPI) {
        double sl = fma(dz, lz, fma(dy, ly, dx * lx));
        double ll = fma(lz, lz, fma(ly, ly, lx * lx));
        float inv = ll > 0.0 ? (float)(1.0 / ll) : 0.0f;
        float pi2 = (float)(sl * sl) * inv;
        float sg2 = fmaxf(v - pi2, 0.0f);
        k1 = guess_lin(__builtin_amdgcn_sqrtf(sg2), P.e1a, P.e1b, P.n1m1);
        k2 = guess_lin(__builtin_amdgcn_sqrtf(pi2), P.e2a, P.e2b, P.n2m1);
    } else {
        k1 = guess1<MODE, EST>(P, v);
        if (MODE == M_RMU_Z) {
            float mu = d2 > 0.0 ? (float)(fabs(dz) / sqrt(d2)) : 0.0f;
            k2 = guess_lin(mu, P.e2a, P.e2b, P.n2m1);
        } else if (MODE == M_RMU_MID) {
            double sl = fma(dz, lz, fma(dy, ly, dx * lx));
            double ll = fma(lz, lz, fma(ly, ly, lx * lx));
            float mu = (d2 > 0.0 && ll > 0.0) ? (float)(fabs(sl) / sqrt(d2 * ll)) : 0.0f;
            k2 = guess_lin(mu, P.e2a, P.e2b, P.n2m1);
        }
    }
    return classify64<MODE>(P, T1, T2, dx, dy, dz, lx, ly, lz, k1, k2);
}

// ---------------------------------------------------------------------------
// FP32 classification with rounding bands.
//
// Bin estimates are kept as biased integers: the bits of the float 2^23 + k.
// The host shifts the estimated variable t by s = (b - 1/2) / a, so that
// fma(t + s, a, 2^23) rounds to 2^23 + floor(t a + b) (for |t a + b| < 2^22);
// the bits are then clamped as unsigned integers to [2^23, 2^23 + n - 1]
// (below 2^23 the float bits are smaller, a NaN or a negative float larger,
// so every estimate lands on a valid index). The low 24 bits are k itself,
// which v_mad_u32_u24 reads directly, and (bits << 3) plus a pre-biased table
// address is the table entry: no float-to-int conversion anywhere.
// Output: in   -> certainly in the estimated bin (same as the canonical decision)
//         out  -> certainly not counted
//         else -> ambiguous (to be re-tested)
// tent: the FP32-only decision (bin or kNoBin), used by FP32_ONLY and for
//       counting flips.
// ---------------------------------------------------------------------------
constexpr uint32_t kBias = 0x4B000000u;   // bits of 2^23

struct C32 {
    bool in, out;
    uint32_t kb, kmb;   // biased estimates of dimension 1 and 2 (kmb = kBias for 1-D kinds)
};

// wave-uniform constants the VALU needs in VGPRs (an fma or med3 can read
// only one SGPR): the bias (which is also the float 2^23) and the LDS
// addresses of the band tables minus the bias times 8
struct Tab32 {
    uint32_t vbias;      // VGPR copy of kBias
    uint32_t tb1, tb2;   // LDS byte address of B1 (B2) - (kBias << 3), modulo 2^32
    float d0;            // VGPR copy of the constant term of the mu band (z line of sight)
};

typedef float __attribute__((ext_vector_type(2))) f2v;
typedef const __attribute__((address_space(3))) f2v* lds_f2p;

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}

template <int EST>
__device__ __forceinline__ Tab32 make_tab32(const CountArgs& P, const float2* B1, const float2* B2) {
    Tab32 t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t.vbias) : "s"(kBias));
    asm volatile("v_mov_b32 %0, %1" : "=v"(t.d0) : "s"(est_muf(EST) ? P.muB0 : P.dA0p));
    t.tb1 = lds_addr(B1) - (kBias << 3);
    t.tb2 = lds_addr(B2) - (kBias << 3);
    return t;
}

__device__ __forceinline__ uint32_t med3u(uint32_t x, uint32_t lo_v, uint32_t hi_s) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo_v), "s"(hi_s));
    return r;
}

// biased estimate from a shifted variable ts (see above)
__device__ __forceinline__ uint32_t est_bits(float ts, float a, const Tab32& T, uint32_t top) {
    return med3u(__float_as_uint(fmaf(ts, a, __uint_as_float(T.vbias))), T.vbias, top);
}

// The same estimate in two parts: the float e = fl(2^23 + x), x = ts a, is
// 2^23 + round(x) for x >= -1/4; its bits clamped to the bins (est_bits) are
// those of the float 2^23 + k, k the pair's bin along that dimension. The
// offset x - k is formed with one rounding (the fma adds 2^23 - (2^23 + k),
// exact, to the exact product ts a): the pair's distance from the centre of
// bin k in bin units, at least 1/2 in size for a pair outside bin k (past
// the first or the last bin included).
__device__ __forceinline__ float est_float(float ts, float a, const Tab32& T) {
    return fmaf(ts, a, __uint_as_float(T.vbias));
}
__device__ __forceinline__ float est_offset(float ts, float a, const Tab32& T, uint32_t kbits) {
    return fmaf(ts, a, __uint_as_float(T.vbias) - __uint_as_float(kbits));
}

// v inside the band [lo, hi'] of its bin (hi' the largest float below the
// upper threshold; an empty band is (inf, inf)): one med3 and one compare,
// whose result is the mask itself
__device__ __forceinline__ bool in_band(float v, float2 b) {
    return __builtin_amdgcn_fmed3f(v, b.x, b.y) == v;
}

__device__ __forceinline__ float2 band_at(uint32_t tb, uint32_t kb) {
    const f2v b = *(lds_f2p)(uintptr_t)((kb << 3) + tb);
    return make_float2(b.x, b.y);
}

// flattened bin of an estimate
__device__ __forceinline__ uint32_t c32_bin(const CountArgs& P, const C32& c) {
    return __umul24(c.kb, (uint32_t)P.n2p1) + (c.kmb - kBias);
}

// LO: the first threshold can be crossed (out_lo >= 0); without it a pair is
// never clean-out on the low side, so that compare is skipped.
template <int MODE, int EST, bool WANT_TENT, bool LO = true>
__device__ __forceinline__ C32 classify32(const CountArgs& P, const Tab32& T, float dx, float dy,
                                          float dz, float lx, float ly, float lz, uint32_t* tent) {
    C32 c;
    c.kmb = kBias;
    float v = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (MODE == M_MONO | MODE == M_THETA) {
        float ts;
        if (MODE == M_THETA) {
            float ch = __builtin_amdgcn_sqrtf(v);
            float th = fmaf(ch * v, 1.0f / 24.0f, ch);  // 2 asin(c/2) to third order
            ts = (est_log(EST) ? __builtin_amdgcn_logf(th) : th) + P.s1;
        } else if (est_log(EST)) {
            ts = __builtin_amdgcn_logf(v) + P.s1;
        } else {
            ts = fmaf(v, __builtin_amdgcn_rsqf(v), P.s1);
        }
        c.kb = est_bits(ts, P.e1a, T, P.top1);
        float2 b = band_at(T.tb1, c.kb);
        c.in = in_band(v, b);
        c.out = LO ? (v >= P.out_hi) | (v < P.out_lo) : (v >= P.out_hi);
        if (WANT_TENT) *tent = (v >= P.bot32 & v < P.top32) ? c.kb - kBias : kNoBin;
        return c;
    }
    if (MODE == M_RMU_Z) {
        float rinv = __builtin_amdgcn_rsqf(v);
        float ts = est_log(EST) ? __builtin_amdgcn_logf(v) + P.s1 : fmaf(v, rinv, P.s1);
        const float er = est_float(ts, P.e1a, T);
        c.kb = med3u(__float_as_uint(er), T.vbias, P.top1);
        float ts2 = fmaf(fabsf(dz), rinv, P.s2);
        const float em = est_float(ts2, P.e2a, T);
        c.kmb = med3u(__float_as_uint(em), T.vbias, P.top2);
        float dz2 = dz * dz;
        // linear r bins: r is decided in bin units as mu is, without the
        // band table; a pair certified there lies inside the v-space band of
        // its bin
        constexpr bool kRx = est_muf(EST) && !est_log(EST) && !WANT_TENT;
        bool rin;
        if constexpr (kRx) {
            rin = fabsf(est_offset(ts, P.e1a, T, c.kb)) <= P.rB0;
        } else {
            float2 b = band_at(T.tb1, c.kb);
            rin = in_band(v, b);
        }
        bool min_;
        if (est_muf(EST) && !WANT_TENT) {
            // in mu space: x = ts2 a = mu a + b - 1/2 is the pair's position
            // in bin units, inside its bin when the offset from the bin's
            // centre is at most 1/2 - beta(r), beta(r) = muB0' + |muB1| / r
            // (T.d0 = 1/2 - muB0', the band kept as a half-width)
            float half = fmaf(P.muB1, rinv, T.d0);
            min_ = fabsf(est_offset(ts2, P.e2a, T, c.kmb)) <= half;
        } else {
            float2 m = band_at(T.tb2, c.kmb);
            // band of the mu predicates, linear in r: dA1 r + dA0. With linear
            // r bins ts = r + s1 and the host folds -dA1 s1 into the constant.
            float delta = est_log(EST) ? fmaf(P.dA1, v * rinv, T.d0) : fmaf(P.dA1, ts, T.d0);
            float flo = fmaf(m.x, v, dz2);
            float fhi = fmaf(m.y, v, dz2);
            min_ = (flo >= delta) & (fhi <= -delta);
        }
        // only r decides a clean "out"; a pair outside a partial mu range is
        // re-tested instead (never the case for mu in [0, 1])
        c.out = LO ? (v >= P.out_hi) | (v < P.out_lo) : (v >= P.out_hi);
        c.in = rin & min_;
        if (WANT_TENT) {
            bool rr = v >= P.bot32 & v < P.top32;
            bool mm = true;
            if (P.d2_partial) mm = (fmaf(P.nlo2_first, v, dz2) >= 0.0f) & (fmaf(P.nhi2_last, v, dz2) < 0.0f);
            *tent = (rr & mm) ? c32_bin(P, c) : kNoBin;
        }
        return c;
    }
    if (MODE == M_RMU_MID) {
        float sl = fmaf(dz, lz, fmaf(dy, ly, dx * lx));
        float ll = fmaf(lz, lz, fmaf(ly, ly, lx * lx));
        float rinv = __builtin_amdgcn_rsqf(v);
        float r = v * rinv;
        float ts = est_log(EST) ? __builtin_amdgcn_logf(v) + P.s1 : r + P.s1;
        c.kb = est_bits(ts, P.e1a, T, P.top1);
        float w = v * ll;
        float sl2 = sl * sl;
        // 1/|l| once: |l| for the band and mu = |s.l| / (r |l|) for the estimate
        float rl = __builtin_amdgcn_rsqf(ll);
        float lnorm = ll * rl;
        c.kmb = est_bits(fmaf(fabsf(sl), rinv * rl, P.s2), P.e2a, T, P.top2);
        float2 b = band_at(T.tb1, c.kb);
        float2 m = band_at(T.tb2, c.kmb);
        float delta = fmaf(ll, fmaf(P.dA2, v, fmaf(P.dA1, r, P.dA0)),
                           fmaf(lnorm, fmaf(P.dB2, v, fmaf(P.dB1, r, P.dB0)),
                                fmaf(P.dC2, v, P.dC0)));
        float flo = fmaf(m.x, w, sl2);
        float fhi = fmaf(m.y, w, sl2);
        bool rin = in_band(v, b);
        bool min_ = (flo >= delta) & (fhi <= -delta);
        c.in = rin & min_ & (ll >= P.llg);
        c.out = LO ? (v >= P.out_hi) | (v < P.out_lo) : (v >= P.out_hi);
        if (WANT_TENT) {
            bool rr = v >= P.bot32 & v < P.top32;
            bool mm = true;
            if (P.d2_partial) mm = (fmaf(P.nlo2_first, w, sl2) >= 0.0f) & (fmaf(P.nhi2_last, w, sl2) < 0.0f);
            *tent = (rr & mm) ? c32_bin(P, c) : kNoBin;
        }
        return c;
    }
    // SIGMAPI (midpoint): sigma^2 ll = |s|^2 |l|^2 - (s.l)^2, pi^2 ll = (s.l)^2
    float sl = fmaf(dz, lz, fmaf(dy, ly, dx * lx));
    float ll = fmaf(lz, lz, fmaf(ly, ly, lx * lx));
    float sl2 = sl * sl;
    float c2 = fmaf(v, ll, -sl2);
    // sigma = sqrt(c2) / |l| and pi = |s.l| / |l| share one 1/|l|. A c2
    // rounded below zero (a pair all but along l) gives a NaN estimate,
    // which the clamp puts in the last sigma bin, whose band test (on c2
    // itself) then fails: the pair is re-tested. The FP32-only decision
    // takes sigma = 0 instead.
    float rl = __builtin_amdgcn_rsqf(ll);
    float sg = __builtin_amdgcn_sqrtf(WANT_TENT ? fmaxf(c2, 0.0f) : c2) * rl;
    float pp = fabsf(sl) * rl;
    c.kb = est_bits(sg + P.s1, P.e1a, T, P.top1);
    c.kmb = est_bits(pp + P.s2, P.e2a, T, P.top2);
    if (WANT_TENT) {
        // out of range: sigma >= sigma_max, pi >= pi_max, or below the first edges
        float fstop = fmaf(P.out_hi, ll, c2);       // out_hi holds -S2f[n1]
        float fptop = fmaf(P.nhi2_last, ll, sl2);   // -P2f[n2]
        float fsbot = fmaf(P.out_lo, ll, c2);       // out_lo holds -S2f[0] (or +BIG)
        float fpbot = fmaf(P.nlo2_first, ll, sl2);  // -P2f[0] (or +BIG)
        bool ok = (fsbot >= 0.0f) & (fstop < 0.0f) & (fpbot >= 0.0f) & (fptop < 0.0f);
        *tent = ok ? c32_bin(P, c) : kNoBin;
        c.in = c.out = false;
        return c;
    }
    // the per-edge parts of the bands are in the tables; the part from the
    // direction error of l is t, in units of F. A bin's entry is (m, H): the
    // pair is inside it along that dimension when |F + m ll| <= H ll - t
    // (F/ll within H - t/ll of the centre -m of the certified interval)
    float t = fmaf(P.spK1, ll * rl, P.spK0);
    float2 bs = band_at(T.tb1, c.kb);
    float2 bp = band_at(T.tb2, c.kmb);
    // |s| below the skip threshold bounds every error term; ll >= llg bounds
    // the direction error of l
    bool vin = v < P.skip32;
    bool lg = ll >= P.llg;
    bool ins = fabsf(fmaf(bs.x, ll, c2)) <= fmaf(bs.y, ll, -t);
    bool inp = fabsf(fmaf(bp.x, ll, sl2)) <= fmaf(bp.y, ll, -t);
    c.in = vin & lg & ins & inp;
    bool top = (fmaf(P.sp_wstop, ll, c2) >= t) | (fmaf(P.sp_wptop, ll, sl2) >= t);
    if (LO) top = top | (fmaf(P.sp_wsbot, ll, c2) <= -t) | (fmaf(P.sp_wpbot, ll, sl2) <= -t);
    c.out = !vin | (lg & top);
    return c;
}

// ---------------------------------------------------------------------------
// Per-wave working state.
// ---------------------------------------------------------------------------
// Periodic image of a neighbour point: (kx+1) | (ky+1) << 2 | (kz+1) << 4,
// k in {-1, 0, 1}; the image lies at q + k L in the home point's frame.
constexpr uint32_t kNoShift = 0x15u;

__device__ __forceinline__ float shift32(uint32_t code, int axis, float Lf) {
    return (float)((int)((code >> (2 * axis)) & 3u) - 1) * Lf;
}
__device__ __forceinline__ double shift64(uint32_t code, int axis, double L) {
    return (double)((int)((code >> (2 * axis)) & 3u) - 1) * L;
}

// Per-wave state. The queue, the histogram and the re-test statistics live
// in LDS; the rare paths take the queue length by value and return it.
struct WaveState {
    unsigned char* hist; // the workgroup's shared histogram (hist_words counters, kH32)
    uint32_t* qi;        // re-test queue: home index
    uint32_t* qj;        // re-test queue: neighbour index
    uint32_t* qc;        // re-test queue: neighbour image code
    unsigned long long* rstat;  // [0] retests, [1] flips (LDS)
    uint32_t tail;       // queued entries (wave-uniform)
    uint64_t evals, tiles;
    // 32-bit histograms: the workgroup's budget of pair evaluations since the
    // histogram was last moved to the global counts (LDS), and this wave's
    // evaluations not reported to it yet
    uint32_t* budget;
    uint32_t pend;
};

// The workgroup's histogram: several interleaved copies so that lanes
// hitting the same bin use different banks, copies a power of two: counter =
// (bin << log2(copies)) | (lane & (copies - 1)). 64-bit counters never wrap;
// 32-bit ones (kH32) are moved to the global counts in time (h32_flush).
template <bool H32>
__device__ __forceinline__ void hist_add(unsigned char* hist, uint32_t bin, int copies, int lane,
                                         uint64_t w = 1u) {
    const uint32_t lc = (uint32_t)__builtin_ctz((unsigned)copies);
    const uint32_t k = (bin << lc) | (uint32_t)(lane & (copies - 1));
    if constexpr (H32)
        atomicAdd(reinterpret_cast<uint32_t*>(hist) + k, (uint32_t)w);
    else
        atomicAdd(reinterpret_cast<unsigned long long*>(hist) + k, (unsigned long long)w);
}

// One increment at an LDS byte address (the lane's copy already folded in).
template <bool H32>
__device__ __forceinline__ void lds_add(uint32_t byte_addr, uint64_t w) {
    if constexpr (H32)
        __hip_atomic_fetch_add((__attribute__((address_space(3))) uint32_t*)(uintptr_t)byte_addr,
                               (uint32_t)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        __hip_atomic_fetch_add((__attribute__((address_space(3))) unsigned long long*)(uintptr_t)byte_addr,
                               (unsigned long long)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Move a 32-bit histogram to the global counts (one wave): every counter is
// swapped with zero, so increments of the other waves land either in the
// value moved or in the emptied counter, and none is lost. Out of line: it
// runs about once per 2^30 increments, and inlined it measured no faster.
__device__ __attribute__((noinline)) void h32_flush(uint32_t* hist, int words, int copies,
                                                    unsigned long long* counts, int lane) {
    const uint32_t lc = (uint32_t)__builtin_ctz((unsigned)copies);
    for (int w = lane; w < words; w += 64) {
        const uint32_t v = atomicExch(&hist[w], 0u);
        if (v) atomicAdd(&counts[(uint32_t)w >> lc], (unsigned long long)v);
    }
}

// Account the pair evaluations of a chunk to the workgroup's budget of a
// 32-bit histogram (every pair adds at most wmax to one counter). A wave
// reports its evaluations every h32_report of them; the wave that finds the
// budget at h32_flush or more resets it and moves the histogram. A counter
// then holds at most h32_flush plus what the waves have not reported or were
// adding during the move (a few h32_report), far below 2^32.
__device__ __forceinline__ void h32_account(const CountArgs& P, WaveState& W, int lane,
                                            uint32_t evals) {
    W.pend += evals;
    if (W.pend < P.h32_report) return;
    uint32_t old = 0;
    if (lane == 0) old = atomicAdd(W.budget, W.pend);
    old = uni(old);
    const uint32_t now = old + W.pend;
    W.pend = 0;
    if (now < P.h32_flush) return;
    if (lane == 0) atomicExch(W.budget, 0u);
    h32_flush(reinterpret_cast<uint32_t*>(W.hist), P.hist_words, P.copies, P.counts, lane);
}

// Weight of a pair in a region pass: wsame if the neighbour lies in the home
// region, wdiff otherwise (1 outside region passes).
__device__ __forceinline__ uint32_t pair_weight(const CountArgs& P, uint32_t j) {
    if (P.regs == nullptr) return 1u;
    return P.regs[j] == (uint16_t)P.region ? P.wsame : P.wdiff;
}

// Weight of the pair (home i, neighbour j): the product of the two point
// weights of pixel maps, else the region weight.
__device__ __forceinline__ uint64_t pair_weight2(const CountArgs& P, uint32_t i, uint32_t j) {
    if (P.wA != nullptr) return (uint64_t)P.wA[i] * (uint64_t)P.wB[j];
    return pair_weight(P, j);
}

// Re-test up to 64 queued pairs per pass, one per lane, through the canonical
// FP64 predicates; count the pairs whose FP32-only decision differs (flips).
// Returns the new queue length.
template <int MODE, int EST>
__device__ __forceinline__ uint32_t drain_queue(
    const CountArgs* __restrict__ Pg, unsigned char* hist, uint32_t* qi, uint32_t* qj, uint32_t* qc,
    unsigned long long* rstat, const float2* B1, const float2* B2, const double* T1,
    const double* T2, int lane, uint32_t tail, bool all) {
    const CountArgs& P = *Pg;
    tail = uni(tail);
    while (tail >= 64u || (all && tail > 0u)) {
        const uint32_t n = tail < 64u ? tail : 64u;
        const bool act = (uint32_t)lane < n;
        uint32_t k = kNoBin, t = kNoBin;
        if (act) {
            const uint32_t i = qi[lane], j = qj[lane], code = qc[lane];
            const P64 p = P.A.p64[i];
            const P64 q = P.B.p64[j];
            k = classify_pair64<MODE, EST>(P, T1, T2, p, q);
            if (k != kNoBin) hist_add<kH32<MODE>>(hist, k, P.copies, lane, pair_weight2(P, i, j));
            // the FP32-only decision of the same pair, as the main loop made it
            const float4 a = P.A.p32[i];
            const float4 b = P.B.p32[j];
            const float Lf = (float)P.L;
            const float qx = b.x - (P.offx - shift32(code, 0, Lf));
            const float qy = b.y - (P.offy - shift32(code, 1, Lf));
            const float qz = b.z - (P.offz - shift32(code, 2, Lf));
            const Tab32 tab = make_tab32<EST>(P, B1, B2);
            (void)classify32<MODE, EST, true>(P, tab, a.x - qx, a.y - qy, a.z - qz,
                                              a.x + (qx + P.lcx), a.y + (qy + P.lcy),
                                              a.z + (qz + P.lcz), &t);
        }
        const uint64_t fl = __builtin_amdgcn_ballot_w64(act && k != t);
        if (lane == 0) {
            rstat[0] += n;
            rstat[1] += (unsigned long long)__popcll(fl);
        }
        const uint32_t rest = tail - n;
        if ((uint32_t)lane < rest) {
            const uint32_t a = qi[n + lane], b = qj[n + lane], c = qc[n + lane];
            qi[lane] = a;
            qj[lane] = b;
            qc[lane] = c;
        }
        tail = rest;
    }
    return tail;
}

// Queue the ambiguous pairs of a chunk: for every home offset o set in hsum,
// the lanes whose bit o is set in ambh (pair: home ts + o, the lane's
// neighbour). Drains whenever 64 or more pairs are waiting. Both functions
// are inlined: most chunks of a clustered catalog queue a pair or two, and an
// out-of-line call costs its argument moves, the registers the call
// convention saves (the r-mu and sigma-pi kernels spilled around it) and a
// stack frame; inlined, the r-mu count takes 3 % less time, the others 1 %.
template <int MODE, int EST>
__device__ __forceinline__ uint32_t enqueue_chunk(
    const CountArgs* __restrict__ Pg, unsigned char* hist, uint32_t* qi, uint32_t* qj, uint32_t* qc,
    unsigned long long* rstat, const float2* B1, const float2* B2, const double* T1,
    const double* T2, int lane, uint32_t tail, uint32_t ts, uint32_t lj, uint32_t lcode,
    uint64_t ambh, uint64_t hsum) {
    tail = uni(tail);
    uint32_t hlo = uni((uint32_t)hsum), hhi = uni((uint32_t)(hsum >> 32));
    while (hlo | hhi) {
        const uint32_t o = hlo ? (uint32_t)__builtin_ctz(hlo) : 32u + (uint32_t)__builtin_ctz(hhi);
        if (o < 32u) hlo &= hlo - 1u; else hhi &= hhi - 1u;
        const bool mine = ((ambh >> o) & 1ull) != 0ull;
        const uint64_t m = __builtin_amdgcn_ballot_w64(mine);
        const uint32_t pre =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (mine) {
            const uint32_t pos = tail + pre;
            qi[pos] = ts + o;
            qj[pos] = lj;
            qc[pos] = lcode;
        }
        tail += (uint32_t)__popcll(m);
        if (tail >= 64u)
            tail = drain_queue<MODE, EST>(Pg, hist, qi, qj, qc, rstat, B1, B2, T1, T2, lane, tail,
                                          false);
    }
    return tail;
}

// ---------------------------------------------------------------------------
// The hot loop. A chunk holds up to 64 neighbour points, one per lane, in
// VGPRs; the home points of the tile are wave-uniform and arrive through
// scalar loads, U at a time, so that U independent pair evaluations per lane
// interleave. Every lane evaluates the pair (home h, its neighbour).
// ---------------------------------------------------------------------------
// Home points h .. h+U-1 not excluded by the point mask (wave-uniform).
template <bool PM, uint32_t U>
__device__ __forceinline__ void home_valid(const CountArgs& P, uint32_t h, bool* hv) {
#pragma unroll
    for (uint32_t u = 0; u < U; u++) hv[u] = true;
    if (PM && P.mbA != nullptr) {
        const cu32p mb = (cu32p)(const void*)P.mbA;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const uint32_t i = h + u;
            hv[u] = ((mb[i >> 5] >> (i & 31u)) & 1u) == 0u;
        }
    }
}

// Every mode has a separation past which no pair is counted: the top edge of
// r or of the chord of theta, the aperture of radial pairs, and for sigma-pi
// sqrt(sigma_max^2 + pi_max^2), since sigma^2 + pi^2 = r^2 for any line of
// sight. A step whose every pair lies past it (skip32 in FP32, on the
// clean-out side of the rounding band; top64 in FP64) is skipped after the
// separations alone. Points are sorted by cell and home tiles are compact, so
// on clustered catalogs whole steps (four home points against a chunk of
// nearby neighbours) often fall beyond r_max together; the separations are
// still formed for every pair.
template <int MODE>
constexpr bool kTopSkip = true;

// Weights of home points h .. h+U-1 (wave-uniform, scalar loads).
template <bool WT, uint32_t U>
__device__ __forceinline__ void home_weights(const CountArgs& P, uint32_t h, uint32_t* hw) {
#pragma unroll
    for (uint32_t u = 0; u < U; u++) hw[u] = 1u;
    if (WT) {
        const cu32p wa = (cu32p)(const void*)P.wA;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) hw[u] = wa[h + u];
    }
}

template <int MODE, int PREC, int EST, bool PM, bool WT, bool MASKED, bool LO, uint32_t U>
__device__ __forceinline__ void step32(const CountArgs& P, WaveState& W, const Tab32& T,
                                       const float2* B1, const float2* B2, const double* T1,
                                       const double* T2, int lane, bool lvalid, bool lmask,
                                       uint32_t lj, uint32_t lcode, float qx, float qy, float qz,
                                       float qlx, float qly, float qlz, uint32_t lb, uint32_t lw,
                                       uint32_t ts, uint64_t& ambh, uint64_t& hsum, uint32_t h) {
    float hx[U], hy[U], hz[U];
    load_points32<U>(P.A.p32, h, hx, hy, hz);
    bool hv[U];
    home_valid<PM, U>(P, h, hv);
    uint32_t hw[U];
    home_weights<WT, U>(P, h, hw);
    if constexpr (kTopSkip<MODE>) {
        // every pair of the step on the clean-out side of the top edge:
        // nothing to count or re-test (see kTopSkip)
        float vmin = 0.f;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const float dx = hx[u] - qx, dy = hy[u] - qy, dz = hz[u] - qz;
            const float v = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            vmin = u == 0 ? v : fminf(vmin, v);
        }
        if (__builtin_amdgcn_ballot_w64(vmin < P.skip32) == 0ull) return;
    }
    uint32_t off[U];
    bool cnt[U], amb[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        const bool act = lvalid & hv[u] &
                         (!MASKED | !lmask | (lj > h + u) | ((P.selfx != 0) & (lj < h + u)));
        const float dx = hx[u] - qx, dy = hy[u] - qy, dz = hz[u] - qz;
        float lx = 0.f, ly = 0.f, lz = 0.f;
        if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
            lx = hx[u] + qlx;
            ly = hy[u] + qly;
            lz = hz[u] + qlz;
        }
        if (PREC == P_FP32O) {
            uint32_t tent;
            (void)classify32<MODE, EST, true>(P, T, dx, dy, dz, lx, ly, lz, &tent);
            cnt[u] = act & (tent != kNoBin);
            off[u] = __umul24(tent, (uint32_t)P.hs2) + lb;
            amb[u] = false;
        } else {
            const C32 c = classify32<MODE, EST, false, LO>(P, T, dx, dy, dz, lx, ly, lz, nullptr);
            cnt[u] = act & c.in;
            amb[u] = act & !(c.in | c.out);
            // LDS byte address of the bin in this lane's copy of the histogram
            if (MODE == M_MONO || MODE == M_THETA)
                off[u] = __umul24(c.kb, (uint32_t)P.hs1) + lb;
            else
                off[u] = __umul24(c.kb, (uint32_t)P.hs1) + (__umul24(c.kmb, (uint32_t)P.hs2) + lb);
        }
    }
    // one vote for the whole step; the per-pair votes only on the rare path
    uint64_t any_amb = 0;
    if (PREC == P_FP32E) {
        bool any = false;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) any = any | amb[u];
        any_amb = __builtin_amdgcn_ballot_w64(any);
    }
#pragma unroll
    for (uint32_t u = 0; u < U; u++)
        if (cnt[u]) lds_add<kH32<MODE>>(off[u], WT ? (uint64_t)lw * hw[u] : (uint64_t)lw);
    if (PREC == P_FP32E && any_amb) {
        // remember the pair for the end of the chunk: bit (home - ts) of this
        // lane's mask, and the home offset in the wave's mask
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const uint64_t bit = 1ull << (h + u - ts);
            if (__builtin_amdgcn_ballot_w64(amb[u])) hsum |= bit;
            if (amb[u]) ambh |= bit;
        }
    }
}

// Radial pairs (Sec. 2.1, radial 2PCF; Sec. 3.4): inside the aperture when
// the chord^2 of the unit vectors is below ap2, then binned by the redshift
// difference |r_i - r_j| against the unsquared edges T1 (half-open).
__device__ __forceinline__ uint32_t classify_radial(const CountArgs& P, const double* T1, double d2,
                                                    double dr) {
    if (!(d2 < P.ap2)) return kNoBin;
    const int n = P.n1;
    if (!(T1[0] <= dr && dr < T1[n])) return kNoBin;
    int lo = 0, hi = n;  // T1[lo] <= dr < T1[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (T1[mid] <= dr) lo = mid; else hi = mid;
    }
    return (uint32_t)lo;
}

template <int MODE, int EST, bool PM, bool WT, bool MASKED, bool SHIFTED, uint32_t U>
__device__ __forceinline__ void step64(const CountArgs& P, WaveState& W, const double* T1,
                                       const double* T2, int lane, bool lvalid, bool lmask,
                                       uint32_t lj, double qx, double qy, double qz, double sx, double sy,
                                       double sz, uint32_t lw, uint32_t h, double qr) {
    double hx[U], hy[U], hz[U];
    load_points64<U>(P.A.p64, h, hx, hy, hz);
    bool hv[U];
    home_valid<PM, U>(P, h, hv);
    uint32_t hw[U];
    home_weights<WT, U>(P, h, hw);
    if constexpr (kTopSkip<MODE>) {
        // every pair of the step at or past the top threshold (exact FP64)
        double dmin = 0.0;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            double dx = hx[u] - qx, dy = hy[u] - qy, dz = hz[u] - qz;
            if (SHIFTED) {
                dx = dx - sx;
                dy = dy - sy;
                dz = dz - sz;
            }
            const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
            dmin = u == 0 ? d2 : fmin(dmin, d2);
        }
        if (__builtin_amdgcn_ballot_w64(dmin < P.top64) == 0ull) return;
    }
    double hr[U];
    if constexpr (MODE == M_RADIAL) {
        const cf64p ra = (cf64p)(const void*)P.rA;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) hr[u] = ra[h + u];
    }
    uint32_t bin[U];
    bool cnt[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        const bool act = lvalid & hv[u] &
                         (!MASKED | !lmask | (lj > h + u) | ((P.selfx != 0) & (lj < h + u)));
        double dx = hx[u] - qx, dy = hy[u] - qy, dz = hz[u] - qz;
        if (SHIFTED) {
            // the neighbour's periodic image: equal to the minimum-image wrap
            // for every pair the stencil can form
            dx = dx - sx;
            dy = dy - sy;
            dz = dz - sz;
        }
        double lx = 0.0, ly = 0.0, lz = 0.0;
        if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
            lx = hx[u] + qx;
            ly = hy[u] + qy;
            lz = hz[u] + qz;
        }
        int k1 = 0, k2 = 0;
        const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if constexpr (MODE == M_RADIAL) {
            bin[u] = classify_radial(P, T1, d2, fabs(hr[u] - qr));
            cnt[u] = act & (bin[u] != kNoBin);
            continue;
        }
        const float v = (float)d2;
        if (MODE == M_MONO || MODE == M_THETA) {
            k1 = guess1<MODE, EST>(P, v);
        } else if (MODE == M_RMU_Z) {
            k1 = guess1<M_MONO, EST>(P, v);
            k2 = guess_lin(fabsf((float)dz) * __builtin_amdgcn_rsqf(v), P.e2a, P.e2b, P.n2m1);
        } else if (MODE == M_RMU_MID) {
            k1 = guess1<M_MONO, EST>(P, v);
            const float sl = (float)fma(dz, lz, fma(dy, ly, dx * lx));
            const float ll = (float)fma(lz, lz, fma(ly, ly, lx * lx));
            k2 = guess_lin(fabsf(sl) * __builtin_amdgcn_rsqf(v * ll), P.e2a, P.e2b, P.n2m1);
        } else {
            const float sl = (float)fma(dz, lz, fma(dy, ly, dx * lx));
            const float ll = (float)fma(lz, lz, fma(ly, ly, lx * lx));
            const float pi2 = sl * sl * __builtin_amdgcn_rcpf(ll);
            k1 = guess_lin(__builtin_amdgcn_sqrtf(fmaxf(v - pi2, 0.0f)), P.e1a, P.e1b, P.n1m1);
            k2 = guess_lin(__builtin_amdgcn_sqrtf(pi2), P.e2a, P.e2b, P.n2m1);
        }
        bin[u] = classify64<MODE>(P, T1, T2, dx, dy, dz, lx, ly, lz, k1, k2);
        cnt[u] = act & (bin[u] != kNoBin);
    }
#pragma unroll
    for (uint32_t u = 0; u < U; u++)
        if (cnt[u]) hist_add<kH32<MODE>>(W.hist, bin[u], P.copies, lane, WT ? (uint64_t)lw * hw[u] : (uint64_t)lw);
}

// The chunk being assembled from neighbour spans (per-lane fields in VGPRs,
// the rest wave-uniform).
struct Chunk {
    uint32_t filled;   // lanes holding a neighbour
    bool masked;       // some lane needs the j > i test
    bool shifted;      // some lane holds a periodic image
    uint32_t lj;       // per lane: neighbour index
    uint32_t lcode;    // per lane: image code
    bool lmask;        // per lane: j > i test applies
};

template <int MODE, int PREC, int EST, bool PM, bool WT>
__device__ void run_chunk(const CountArgs& P, WaveState& W, const float2* B1, const float2* B2,
                          const double* T1, const double* T2, int lane, Chunk& C, uint32_t ts,
                          uint32_t te) {
    constexpr uint32_t U = 4;
    if constexpr (kH32<MODE>) {
        // every pair of the chunk adds at most the largest region weight
        const uint32_t wmax = P.regs == nullptr ? 1u : (P.wsame > P.wdiff ? P.wsame : P.wdiff);
        h32_account(P, W, lane, C.filled * (te - ts) * wmax);
    }
    bool lvalid = (uint32_t)lane < C.filled;
    // a neighbour excluded by the point mask leaves its lane idle
    if (PM && P.mbB != nullptr && lvalid) lvalid = ((P.mbB[C.lj >> 5] >> (C.lj & 31u)) & 1u) == 0u;
    const uint32_t lw = lvalid ? (WT ? P.wB[C.lj] : pair_weight(P, C.lj)) : 1u;
    if constexpr (PREC == P_FP64) {
        double qx = 0.0, qy = 0.0, qz = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, qr = 0.0;
        if (MODE == M_RADIAL && lvalid) qr = P.rB[C.lj];
        if (lvalid) {
            const P64 q = P.B.p64[C.lj];
            qx = q.x;
            qy = q.y;
            qz = q.z;
            sx = shift64(C.lcode, 0, P.L);
            sy = shift64(C.lcode, 1, P.L);
            sz = shift64(C.lcode, 2, P.L);
        }
#define CUTE_RUN64(MSK, SH)                                                                     \
    {                                                                                           \
        uint32_t h = ts;                                                                        \
        for (; h + U <= te; h += U)                                                             \
            step64<MODE, EST, PM, WT, MSK, SH, U>(P, W, T1, T2, lane, lvalid, C.lmask, C.lj, qx, qy, qz, \
                                          sx, sy, sz, lw, h, qr);                               \
        for (; h < te; h++)                                                                     \
            step64<MODE, EST, PM, WT, MSK, SH, 1>(P, W, T1, T2, lane, lvalid, C.lmask, C.lj, qx, qy, qz, \
                                          sx, sy, sz, lw, h, qr);                               \
    }
        if (C.masked) {
            if (C.shifted) CUTE_RUN64(true, true) else CUTE_RUN64(true, false)
        } else {
            if (C.shifted) CUTE_RUN64(false, true) else CUTE_RUN64(false, false)
        }
#undef CUTE_RUN64
    } else {
        // wave-uniform constants in VGPRs, and this lane's histogram copy
        const Tab32 tab = make_tab32<EST>(P, B1, B2);
        const uint32_t lb = lds_addr(W.hist) +
                            ((uint32_t)lane & (uint32_t)(P.copies - 1)) * (kH32<MODE> ? 4u : 8u);
        // the neighbour in the home grid's FP32 frame: q - (cA - cB) for two
        // open grids, or its periodic image q + k L (only one of the two is
        // ever non-zero), and q + 2 cA for the midpoint line of sight
        float qx = 0.f, qy = 0.f, qz = 0.f, qlx = 0.f, qly = 0.f, qlz = 0.f;
        if (lvalid) {
            const float4 q = P.B.p32[C.lj];
            const float Lf = (float)P.L;
            qx = q.x - (P.offx - shift32(C.lcode, 0, Lf));
            qy = q.y - (P.offy - shift32(C.lcode, 1, Lf));
            qz = q.z - (P.offz - shift32(C.lcode, 2, Lf));
            qlx = qx + P.lcx;
            qly = qy + P.lcy;
            qlz = qz + P.lcz;
        }
#define CUTE_RUN32(MSK, LOW)                                                                     \
    {                                                                                              \
        uint32_t h = ts;                                                                           \
        for (; h + U <= te; h += U)                                                                \
            step32<MODE, PREC, EST, PM, WT, MSK, LOW, U>(P, W, tab, B1, B2, T1, T2, lane, lvalid,  \
                                                     C.lmask, C.lj, C.lcode, qx, qy, qz, qlx, qly, \
                                                     qlz, lb, lw, ts, ambh, hsum, h);              \
        for (; h < te; h++)                                                                        \
            step32<MODE, PREC, EST, PM, WT, MSK, LOW, 1>(P, W, tab, B1, B2, T1, T2, lane, lvalid,  \
                                                     C.lmask, C.lj, C.lcode, qx, qy, qz, qlx, qly, \
                                                     qlz, lb, lw, ts, ambh, hsum, h);              \
    }
        // ambiguous pairs of this chunk: per lane, bit (home - ts); per wave,
        // the home offsets with any (queued once the home loop is done)
        uint64_t ambh = 0, hsum = 0;
        // bins starting at zero separation have no low-side clean "out"
        const bool low = MODE == M_SIGMAPI ? P.sp_low != 0 : !(P.out_lo < 0.0f);
        if (C.masked) {
            if (low) CUTE_RUN32(true, true) else CUTE_RUN32(true, false)
        } else {
            if (low) CUTE_RUN32(false, true) else CUTE_RUN32(false, false)
        }
        if (PREC == P_FP32E && hsum != 0ull)
            W.tail = enqueue_chunk<MODE, EST>(P.self, W.hist, W.qi, W.qj, W.qc, W.rstat, B1, B2, T1,
                                              T2, lane, W.tail, ts, C.lj, C.lcode, ambh, hsum);
#undef CUTE_RUN32
    }
    C.filled = 0;
    C.masked = false;
    C.shifted = false;
}

// Append the neighbour span [a0, a1) (image code, j > i test) to the chunk,
// running every chunk that fills up.
template <int MODE, int PREC, int EST, bool PM, bool WT>
__device__ void feed(const CountArgs& P, WaveState& W, const float2* B1, const float2* B2,
                     const double* T1, const double* T2, int lane, Chunk& C, uint32_t ts,
                     uint32_t te, uint32_t a0, uint32_t a1, uint32_t code, bool masked) {
    if (masked && a1 > a0 && P.selfx) {
        // the tile against itself: every pair but the point with itself
        W.evals += (uint64_t)(te - ts) * (a1 - a0) - (a1 - a0);
    } else if (masked && a1 > a0) {
        // lanes with neighbour j pair with the home points h < j: sum of (j - ts)
        const uint64_t lo_ = a0 - ts, hi_ = a1 - 1u - ts;
        W.evals += (lo_ + hi_) * (hi_ - lo_ + 1u) / 2u;
    } else if (a1 > a0) {
        W.evals += (uint64_t)(te - ts) * (a1 - a0);
    }
    while (a0 < a1) {
        const uint32_t room = 64u - C.filled;
        const uint32_t take = (a1 - a0) < room ? (a1 - a0) : room;
        const uint32_t l = (uint32_t)lane;
        if (l >= C.filled && l < C.filled + take) {
            C.lj = a0 + (l - C.filled);
            C.lcode = code;
            C.lmask = masked;
        }
        C.filled += take;
        C.masked = C.masked | masked;
        C.shifted = C.shifted | (code != kNoShift);
        a0 += take;
        if (C.filled == 64u) run_chunk<MODE, PREC, EST, PM, WT>(P, W, B1, B2, T1, T2, lane, C, ts, te);
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ int imod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Span list of one tile, built in LDS before any pair is evaluated, so that
// the stencil's FP64 temporaries are dead while the hot loop runs.
struct SpanBuf {
    uint32_t* a;   // first neighbour index
    uint32_t* b;   // one past the last
    uint32_t* f;   // image code (low 8 bits) | j > i test (bit 8)
    uint32_t n;    // entries (wave-uniform)
};

__device__ __forceinline__ void push_span(SpanBuf& S, int lane, uint32_t a0, uint32_t a1,
                                          uint32_t code, bool masked) {
    if (a1 <= a0) return;
    if (lane == 0) {
        S.a[S.n] = a0;
        S.b[S.n] = a1;
        S.f[S.n] = code | (masked ? 0x100u : 0u);
    }
    S.n++;
}

// Neighbour spans of the cell range [pa, pb] of row rb in the B grid. In the
// home row of an autocorrelation the range starting at the tile's first cell
// is split into the tile itself (pairs j > i only) and the rest.
__device__ __forceinline__ void push_cells(SpanBuf& S, int lane, const cu32p cs, uint32_t rb,
                                           int pa, int pb, uint32_t code, bool home_start,
                                           uint32_t ts, uint32_t te) {
    const uint32_t j0 = uni(cs[rb + (uint32_t)pa]);
    const uint32_t j1 = uni(cs[rb + (uint32_t)pb + 1u]);
    if (home_start) {
        // points of the first cell before the tile pair with it from their own tile
        const uint32_t m1 = te < j1 ? te : j1;
        push_span(S, lane, ts, m1, code, true);
        push_span(S, lane, m1 > te ? m1 : te, j1, code, false);
    } else {
        push_span(S, lane, j0, j1, code, false);
    }
}

// Fill the span buffer with the neighbour spans of rows [*row, ...) of the
// tile's stencil (Sec. 3.3: the cells within r_max of the tile), stopping
// before the buffer could overflow. Returns true when every row is done.
__device__ bool gen_spans(const CountArgs& P, const Tile& tl, int lane, SpanBuf& S, int* row) {
    const uint32_t ts = tl.start, te = tl.end;
    const int c0 = (int)(tl.c0c1 & 0xffffu), c1 = (int)(tl.c0c1 >> 16);
    const GridView& A = P.A;
    const GridView& B = P.B;
    const int cy = (int)(tl.row % (uint32_t)A.ny), cz = (int)(tl.row / (uint32_t)A.ny);
    const cu32p cs = (cu32p)(const void*)B.cstart;
    S.n = 0;
    const uint32_t room = kSpanCap - 3;

    if (P.geom == CUTE_GEOM_SPHERE) {
        // tile pixel block: phi in [c0, c1+1) * ax, cos theta in one band
        const double zlo = A.oy + cy * A.ay, zhi = zlo + A.ay;
        const double zl = fmax(-1.0, fmin(1.0, zlo)), zh = fmax(-1.0, fmin(1.0, zhi));
        const double th_lo = acos(zh), th_hi = acos(zl);
        const double ths = P.th_s;
        const double zn_hi = (th_lo - ths <= 0.0) ? 1.0 : cos(th_lo - ths);
        const double zn_lo = (th_hi + ths >= kPi) ? -1.0 : cos(th_hi + ths);
        int b0 = (int)floor((zn_lo - B.oy) / B.ay) - 1, b1 = (int)floor((zn_hi - B.oy) / B.ay) + 1;
        b0 = clampi(b0, 0, B.ny - 1);
        b1 = clampi(b1, 0, B.ny - 1);
        // half-width in phi of a cap of radius th_s around any tile point:
        // asin(sin th_s / sin theta) at the tile colatitude nearest a pole
        const double zmax2 = fmax(zl * zl, zh * zh);
        const double smin = sqrt(fmax(0.0, 1.0 - zmax2));
        bool full = !(P.sin_th_s < smin * (1.0 - 1e-9)) || (P.th_s >= 0.5 * kPi);
        const double hw = full ? 0.0 : asin(P.sin_th_s / smin) * (1.0 + 1e-9) + 1e-12;
        const double phlo = c0 * A.ax - hw, phhi = (c1 + 1) * A.ax + hw;
        const int x0 = (int)floor(phlo / B.ax) - 1, x1 = (int)floor(phhi / B.ax) + 1;
        if (x1 - x0 + 1 >= B.nx) full = true;
        for (int by = b0 + *row; by <= b1; by++) {
            if (S.n > room) {
                *row = by - b0;
                return false;
            }
            const int byu = unii(by);
            const bool same = P.is_auto && byu == cy;
            if (P.is_auto && byu < cy) continue;
            const uint32_t rb = (uint32_t)byu * (uint32_t)B.nx;
            if (same) {
                // index rule inside the home band: partners with a larger
                // index, i.e. cells >= c0 up to the right reach, plus the left
                // reach that wraps past phi = 2 pi onto the band's last cells
                int p0b = B.nx - 1, p1a = 0, p1b = -1;
                if (!full) {
                    const int r1 = x1 < B.nx - 1 ? x1 : B.nx - 1;
                    const int s2 = x0 < 0 ? x0 + B.nx : B.nx;
                    if (s2 > r1 + 1) {
                        p0b = r1;
                        p1a = s2;
                        p1b = B.nx - 1;
                    }
                }
                push_cells(S, lane, cs, rb, c0, p0b, kNoShift, true, ts, te);
                if (p1b >= p1a) push_cells(S, lane, cs, rb, p1a, p1b, kNoShift, false, ts, te);
            } else if (full) {
                push_cells(S, lane, cs, rb, 0, B.nx - 1, kNoShift, false, ts, te);
            } else {
                // cyclic range [x0, x1] (length < nx) split at the phi wrap
                const int a0 = imod(x0, B.nx);
                const int len = x1 - x0 + 1;
                if (a0 + len <= B.nx) {
                    push_cells(S, lane, cs, rb, a0, a0 + len - 1, kNoShift, false, ts, te);
                } else {
                    push_cells(S, lane, cs, rb, a0, B.nx - 1, kNoShift, false, ts, te);
                    push_cells(S, lane, cs, rb, 0, a0 + len - 1 - B.nx, kNoShift, false, ts, te);
                }
            }
        }
        return true;
    }

    // 3-D boxes of one geometry: the rows are precomputed offsets
    if (P.stencil != nullptr) {
        const cu32p st = (cu32p)(const void*)P.stencil;
        for (int e = *row; e < P.nst; e++) {
            if (S.n > room) {
                *row = e;
                return false;
            }
            const int ody = (int)uni(st[4 * e]), odz = (int)uni(st[4 * e + 1]);
            const int left = (int)uni(st[4 * e + 2]), right = (int)uni(st[4 * e + 3]);
            const int byu = cy + ody, bzu = cz + odz;
            const bool same = P.is_auto && ody == 0 && odz == 0;
            const bool home = P.selfx && ody == 0 && odz == 0;
            int x0 = same ? c0 : c0 - left, x1 = c1 + right;
            int ry = byu, rz = bzu, ky = 0, kz = 0;
            if (P.periodic) {
                ky = floordiv(byu, B.ny);
                kz = floordiv(bzu, B.nz);
                ry = byu - ky * B.ny;
                rz = bzu - kz * B.nz;
                // never more than one full turn of the row
                x1 = x1 < x0 + B.nx - 1 ? x1 : x0 + B.nx - 1;
            } else {
                if (byu < 0 || byu >= B.ny || bzu < 0 || bzu >= B.nz) continue;
                x0 = x0 < 0 ? 0 : x0;
                x1 = x1 > B.nx - 1 ? B.nx - 1 : x1;
                if (x0 > x1) continue;
            }
            const uint32_t rb = (uint32_t)B.nx * ((uint32_t)ry + (uint32_t)B.ny * (uint32_t)rz);
            int a0 = x0;
            while (a0 <= x1) {
                const int kx = P.periodic ? floordiv(a0, B.nx) : 0;
                const int lim = P.periodic ? (kx + 1) * B.nx - 1 : x1;
                const int a1 = x1 < lim ? x1 : lim;
                const uint32_t code =
                    (uint32_t)(kx + 1) | ((uint32_t)(ky + 1) << 2) | ((uint32_t)(kz + 1) << 4);
                if (home && kx == 0 && a0 <= c0 && c1 <= a1) {
                    // full stencil over one catalog: the tile's own cells are
                    // split around the tile, whose points pair with all but
                    // themselves (the j != i test)
                    if (a0 < c0) push_cells(S, lane, cs, rb, a0, c0 - 1, code, false, ts, te);
                    const uint32_t j0 = uni(cs[rb + (uint32_t)c0]);
                    const uint32_t j1 = uni(cs[rb + (uint32_t)c1 + 1u]);
                    push_span(S, lane, j0, ts, code, false);
                    push_span(S, lane, ts, te, code, true);
                    push_span(S, lane, te, j1, code, false);
                    if (c1 < a1) push_cells(S, lane, cs, rb, c1 + 1, a1, code, false, ts, te);
                } else {
                    push_cells(S, lane, cs, rb, a0 - kx * B.nx, a1 - kx * B.nx, code,
                               same && kx == 0 && a0 == c0, ts, te);
                }
                a0 = a1 + 1;
            }
        }
        return true;
    }

    // 3-D boxes: the tile box, grown by R, selects rows of neighbour cells
    const double R = P.Rs;
    const double xlo = A.ox + c0 * A.ax, xhi = A.ox + (c1 + 1) * A.ax;
    const double ylo = A.oy + cy * A.ay, yhi = ylo + A.ay;
    const double zlo = A.oz + cz * A.az, zhi = zlo + A.az;
    int y0 = (int)floor((ylo - R - B.oy) / B.ay), y1 = (int)floor((yhi + R - B.oy) / B.ay);
    int z0 = (int)floor((zlo - R - B.oz) / B.az), z1 = (int)floor((zhi + R - B.oz) / B.az);
    if (!P.periodic) {
        y0 = clampi(y0, 0, B.ny - 1);
        y1 = clampi(y1, 0, B.ny - 1);
        z0 = clampi(z0, 0, B.nz - 1);
        z1 = clampi(z1, 0, B.nz - 1);
    }
    const int nyr = y1 - y0 + 1;
    const int nrows = nyr * (z1 - z0 + 1);
    const double R2 = R * R;
    for (int r = *row; r < nrows; r++) {
        if (S.n > room) {
            *row = r;
            return false;
        }
        const int bzu = unii(z0 + r / nyr), byu = unii(y0 + r % nyr);
        bool same = false;
        if (P.is_auto) {
            const int oz_ = bzu - cz, oy_ = byu - cy;
            if (oz_ < 0 || (oz_ == 0 && oy_ < 0)) continue;
            same = (oz_ == 0 && oy_ == 0);
        }
        // distance in y and z between the tile box and this row of cells
        const double rylo = B.oy + byu * B.ay, ryhi = rylo + B.ay;
        const double rzlo = B.oz + bzu * B.az, rzhi = rzlo + B.az;
        const double dy = fmax(0.0, fmax(rylo - yhi, ylo - ryhi));
        const double dz = fmax(0.0, fmax(rzlo - zhi, zlo - rzhi));
        const double rem = R2 - dy * dy - dz * dz;
        if (rem <= 0.0) continue;
        const double w = sqrt(rem);
        int x0 = (int)floor((xlo - w - B.ox) / B.ax), x1 = (int)floor((xhi + w - B.ox) / B.ax);
        if (same && x0 < c0) x0 = c0;
        int ry = byu, rz = bzu, ky = 0, kz = 0;
        if (P.periodic) {
            ky = floordiv(byu, B.ny);
            kz = floordiv(bzu, B.nz);
            ry = byu - ky * B.ny;
            rz = bzu - kz * B.nz;
        } else {
            x0 = x0 < 0 ? 0 : x0;
            x1 = x1 > B.nx - 1 ? B.nx - 1 : x1;
            if (x0 > x1) continue;
        }
        const uint32_t rb = (uint32_t)B.nx * ((uint32_t)ry + (uint32_t)B.ny * (uint32_t)rz);
        // split [x0, x1] at periodic wraps (at most two pieces)
        int a0 = x0;
        while (a0 <= x1) {
            const int kx = P.periodic ? floordiv(a0, B.nx) : 0;
            const int lim = P.periodic ? (kx + 1) * B.nx - 1 : x1;
            const int a1 = x1 < lim ? x1 : lim;
            const uint32_t code =
                (uint32_t)(kx + 1) | ((uint32_t)(ky + 1) << 2) | ((uint32_t)(kz + 1) << 4);
            push_cells(S, lane, cs, rb, a0 - kx * B.nx, a1 - kx * B.nx, code,
                       same && kx == 0 && a0 == c0, ts, te);
            a0 = a1 + 1;
        }
    }
    return true;
}

// Count the pairs of one home tile: spans are generated into the LDS span
// buffer, then fed chunk by chunk to the hot loop.
template <int MODE, int PREC, int EST, bool PM, bool WT>
__device__ void do_tile(const CountArgs& P, WaveState& W, SpanBuf& S, const float2* B1,
                        const float2* B2, const double* T1, const double* T2, int lane,
                        const Tile& tl) {
    W.tiles++;
    if (PM && P.mbA != nullptr) {
        // a tile whose home points are all masked out has no pair to count
        const uint32_t i = tl.start + (uint32_t)lane;
        const bool live = i < tl.end && ((P.mbA[i >> 5] >> (i & 31u)) & 1u) == 0u;
        if (__builtin_amdgcn_ballot_w64(live) == 0ull) return;
    }
    Chunk C;
    C.filled = 0;
    C.masked = false;
    C.shifted = false;
    C.lj = 0;
    C.lcode = kNoShift;
    C.lmask = false;
    int row = 0;
    bool done = false;
    while (!done) {
        done = gen_spans(P, tl, lane, S, &row);
        for (uint32_t k = 0; k < S.n; k++) {
            const uint32_t a0 = uni(S.a[k]), a1 = uni(S.b[k]), f = uni(S.f[k]);
            feed<MODE, PREC, EST, PM, WT>(P, W, B1, B2, T1, T2, lane, C, tl.start, tl.end, a0, a1,
                                  f & 0xffu, (f & 0x100u) != 0u);
        }
    }
    if (C.filled) run_chunk<MODE, PREC, EST, PM, WT>(P, W, B1, B2, T1, T2, lane, C, tl.start, tl.end);
}


}  // namespace
}  // namespace cute
