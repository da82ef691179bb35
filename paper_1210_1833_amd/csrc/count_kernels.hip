// Pair-count kernels for gfx950.
//
// One wavefront owns one home tile at a time (a run of up to 64 sorted points
// inside one row of cells, one point per lane) and walks the neighbour cells
// of Sec. 3.3 as contiguous spans of the other catalog. The neighbour point
// is wave-uniform, so its coordinates arrive through scalar loads and enter
// the VALU as scalar operands; every lane evaluates its own pair. Counts go
// to a per-wave LDS histogram (several interleaved copies, one per lane
// group, so that lanes hitting the same bin use different banks) and are
// flushed into uint64 global counts.
//
// Precision paths
//  - FP64: every pair is classified by the canonical FP64 predicates.
//  - FP32_EDGE: separations in FP32; a pair is counted directly only when its
//    FP32 value is farther than a proven rounding bound from every decision
//    threshold (bin edges, r_max, mu edges); the rest go to a per-wave LDS
//    queue that is drained 64 pairs at a time through the canonical FP64
//    predicates, so the counts equal the FP64 ones.
//  - FP32_ONLY: FP32 decisions only.
#include <math.h>
#include <stdint.h>

#include "cute_internal.h"
#include "runtime.h"

namespace cute {

namespace {

constexpr int kQCap = 128;             // retest queue entries per wave
constexpr uint32_t kNoBin = 0xffffffffu;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr uint32_t kChunk = 1u << 20;  // neighbour points per budget check

// Read-only device memory seen through the constant address space: loads at
// wave-uniform addresses become scalar (s_load) loads into SGPRs.
typedef const __attribute__((address_space(4))) float* cfp;
typedef const __attribute__((address_space(4))) double* cdp;
typedef const __attribute__((address_space(4))) uint32_t* cu32p;

__device__ __forceinline__ float4 load_u32x4f(const float4* p, uint32_t j) {
    const cfp f = (cfp)(const void*)p;
    return make_float4(f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3]);
}
__device__ __forceinline__ P64 load_u64x3(const P64* p, uint32_t j) {
    const cdp f = (cdp)(const void*)p;
    P64 q;
    q.x = f[4 * j];
    q.y = f[4 * j + 1];
    q.z = f[4 * j + 2];
    q.w = 0.0;
    return q;
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
        t = (EST == E_LOG) ? __builtin_amdgcn_logf(th) : th;
    } else {
        t = (EST == E_LOG) ? __builtin_amdgcn_logf(v) : __builtin_amdgcn_sqrtf(v);
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
// Output: in   -> certainly in bin *bin (same as the canonical decision)
//         out  -> certainly not counted
//         else -> ambiguous (to be re-tested); *bin holds the FP32 guess
// tent: the FP32-only decision (bin or kNoBin), used by FP32_ONLY and for
//       counting flips.
// ---------------------------------------------------------------------------
struct C32 {
    bool in, out;
    uint32_t bin;
};

template <int MODE, int EST, bool WANT_TENT>
__device__ __forceinline__ C32 classify32(const CountArgs& P, const float2* B1,
                                          const float2* B2, float dx, float dy, float dz,
                                          float lx, float ly, float lz, uint32_t* tent) {
    C32 c;
    float v = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (MODE == M_MONO | MODE == M_THETA) {
        int k = guess1<MODE, EST>(P, v);
        float2 b = B1[k];
        c.in = (v >= b.x) & (v < b.y);
        c.out = (v >= P.out_hi) | (v < P.out_lo);
        c.bin = (uint32_t)k;
        if (WANT_TENT) *tent = (v >= P.bot32 & v < P.top32) ? (uint32_t)k : kNoBin;
        return c;
    }
    if (MODE == M_RMU_Z) {
        float rinv = __builtin_amdgcn_rsqf(v);
        float r = v * rinv;
        int k;
        if (EST == E_LOG) {
            k = guess_lin(__builtin_amdgcn_logf(v), P.e1a, P.e1b, P.n1m1);
        } else {
            k = guess_lin(r, P.e1a, P.e1b, P.n1m1);
        }
        float mu = fabsf(dz) * rinv;
        int km = guess_lin(mu, P.e2a, P.e2b, P.n2m1);
        float dz2 = dz * dz;
        float2 b = B1[k];
        float2 m = B2[km];
        float delta = fmaf(P.dA2, v, fmaf(P.dA1, r, P.dA0));
        float flo = fmaf(m.x, v, dz2);
        float fhi = fmaf(m.y, v, dz2);
        bool rin = (v >= b.x) & (v < b.y);
        bool min_ = (flo >= delta) & (fhi <= -delta);
        c.in = rin & min_;
        // only r decides a clean "out"; a pair outside a partial mu range is
        // re-tested instead (never the case for mu in [0, 1])
        c.out = (v >= P.out_hi) | (v < P.out_lo);
        c.bin = __umul24((uint32_t)k, (uint32_t)P.n2) + (uint32_t)km;
        if (WANT_TENT) {
            bool rr = v >= P.bot32 & v < P.top32;
            bool mm = true;
            if (P.d2_partial) mm = (fmaf(P.nlo2_first, v, dz2) >= 0.0f) & (fmaf(P.nhi2_last, v, dz2) < 0.0f);
            *tent = (rr & mm) ? c.bin : kNoBin;
        }
        return c;
    }
    if (MODE == M_RMU_MID) {
        float sl = fmaf(dz, lz, fmaf(dy, ly, dx * lx));
        float ll = fmaf(lz, lz, fmaf(ly, ly, lx * lx));
        float rinv = __builtin_amdgcn_rsqf(v);
        float r = v * rinv;
        int k = (EST == E_LOG) ? guess_lin(__builtin_amdgcn_logf(v), P.e1a, P.e1b, P.n1m1)
                               : guess_lin(r, P.e1a, P.e1b, P.n1m1);
        float w = v * ll;
        float sl2 = sl * sl;
        float lnorm = __builtin_amdgcn_sqrtf(ll);
        float mu = fabsf(sl) * rinv * __builtin_amdgcn_rcpf(lnorm);
        int km = guess_lin(mu, P.e2a, P.e2b, P.n2m1);
        float2 b = B1[k];
        float2 m = B2[km];
        float delta = fmaf(ll, fmaf(P.dA2, v, fmaf(P.dA1, r, P.dA0)),
                           fmaf(lnorm, fmaf(P.dB2, v, fmaf(P.dB1, r, P.dB0)),
                                fmaf(P.dC2, v, P.dC0)));
        float flo = fmaf(m.x, w, sl2);
        float fhi = fmaf(m.y, w, sl2);
        bool rin = (v >= b.x) & (v < b.y);
        bool min_ = (flo >= delta) & (fhi <= -delta);
        c.in = rin & min_;
        c.out = (v >= P.out_hi) | (v < P.out_lo);
        c.bin = __umul24((uint32_t)k, (uint32_t)P.n2) + (uint32_t)km;
        if (WANT_TENT) {
            bool rr = v >= P.bot32 & v < P.top32;
            bool mm = true;
            if (P.d2_partial) mm = (fmaf(P.nlo2_first, w, sl2) >= 0.0f) & (fmaf(P.nhi2_last, w, sl2) < 0.0f);
            *tent = (rr & mm) ? c.bin : kNoBin;
        }
        return c;
    }
    // SIGMAPI (midpoint): sigma^2 ll = |s|^2 |l|^2 - (s.l)^2, pi^2 ll = (s.l)^2
    float sl = fmaf(dz, lz, fmaf(dy, ly, dx * lx));
    float ll = fmaf(lz, lz, fmaf(ly, ly, lx * lx));
    float sl2 = sl * sl;
    float c2 = fmaf(v, ll, -sl2);
    float rll = __builtin_amdgcn_rcpf(ll);
    float sg = __builtin_amdgcn_sqrtf(fmaxf(c2 * rll, 0.0f));
    float pp = __builtin_amdgcn_sqrtf(sl2 * rll);
    int ks = guess_lin(sg, P.e1a, P.e1b, P.n1m1);
    int kp = guess_lin(pp, P.e2a, P.e2b, P.n2m1);
    float t = __builtin_amdgcn_sqrtf(v);
    float lnorm = __builtin_amdgcn_sqrtf(ll);
    float ds = fmaf(ll, fmaf(P.sA2, v, fmaf(P.sA1, t, P.sA0)),
                    fmaf(lnorm, fmaf(P.sB2, v, fmaf(P.sB1, t, P.sB0)), fmaf(P.sC2, v, P.sC0)));
    float dp = fmaf(ll, fmaf(P.dA2, v, fmaf(P.dA1, t, P.dA0)),
                    fmaf(lnorm, fmaf(P.dB2, v, fmaf(P.dB1, t, P.dB0)), fmaf(P.dC2, v, P.dC0)));
    float2 bs = B1[ks];
    float2 bp = B2[kp];
    float fslo = fmaf(bs.x, ll, c2), fshi = fmaf(bs.y, ll, c2);
    float fplo = fmaf(bp.x, ll, sl2), fphi = fmaf(bp.y, ll, sl2);
    c.in = (fslo >= ds) & (fshi <= -ds) & (fplo >= dp) & (fphi <= -dp);
    // out of range: sigma >= sigma_max, pi >= pi_max, or below the first edges
    float fstop = fmaf(P.out_hi, ll, c2);       // out_hi holds -S2f[n1]
    float fptop = fmaf(P.nhi2_last, ll, sl2);   // -P2f[n2]
    float fsbot = fmaf(P.out_lo, ll, c2);       // out_lo holds -S2f[0] (or +BIG)
    float fpbot = fmaf(P.nlo2_first, ll, sl2);  // -P2f[0] (or +BIG)
    c.out = (fstop >= ds) | (fptop >= dp) | (fsbot <= -ds) | (fpbot <= -dp);
    c.bin = __umul24((uint32_t)ks, (uint32_t)P.n2) + (uint32_t)kp;
    if (WANT_TENT) {
        bool ok = (fsbot >= 0.0f) & (fstop < 0.0f) & (fpbot >= 0.0f) & (fptop < 0.0f);
        *tent = ok ? c.bin : kNoBin;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Per-wave working state.
// ---------------------------------------------------------------------------
struct WaveState {
    uint32_t* hist;      // hist_words words
    uint32_t* qi;        // queue: home index
    uint32_t* qj;        // queue: neighbour index
    uint32_t* qt;        // queue: FP32 decision
    uint32_t tail;       // queued entries (wave-uniform)
    uint64_t since_flush;
    uint64_t evals, retests, flips, tiles;
};

// copies is a power of two: word = (bin << log2(copies)) | (lane & (copies - 1))
__device__ __forceinline__ void hist_add(uint32_t* hist, uint32_t bin, int copies, int lane) {
    const uint32_t lc = (uint32_t)__builtin_ctz((unsigned)copies);
    atomicAdd(&hist[(bin << lc) | (uint32_t)(lane & (copies - 1))], 1u);
}

template <int MODE, int EST>
__device__ void drain_queue(const CountArgs& P, WaveState& W, const double* T1, const double* T2,
                            int lane, bool all) {
    while (W.tail >= 64u || (all && W.tail > 0u)) {
        const uint32_t n = W.tail < 64u ? W.tail : 64u;
        const bool act = (uint32_t)lane < n;
        uint32_t k = kNoBin, t = kNoBin;
        if (act) {
            const uint32_t i = W.qi[lane], j = W.qj[lane];
            t = W.qt[lane];
            const P64 p = P.A.p64[i];
            const P64 q = P.B.p64[j];
            k = classify_pair64<MODE, EST>(P, T1, T2, p, q);
            if (k != kNoBin) hist_add(W.hist, k, P.copies, lane);
        }
        const uint64_t fl = __builtin_amdgcn_ballot_w64(act && k != t);
        W.flips += (uint64_t)__popcll(fl);
        W.retests += n;
        const uint32_t rest = W.tail - n;
        if ((uint32_t)lane < rest) {
            const uint32_t a = W.qi[n + lane], b = W.qj[n + lane], c = W.qt[n + lane];
            W.qi[lane] = a;
            W.qj[lane] = b;
            W.qt[lane] = c;
        }
        W.tail = rest;
    }
}

template <int MODE, int EST>
__device__ void wave_flush(const CountArgs& P, WaveState& W, const double* T1, const double* T2,
                           int lane) {
    drain_queue<MODE, EST>(P, W, T1, T2, lane, true);
    for (int b = lane; b < P.nbins; b += 64) {
        uint64_t s = 0;
        for (int c = 0; c < P.copies; c++) {
            uint32_t* w = &W.hist[b * P.copies + c];
            s += *w;
            *w = 0u;
        }
        if (s) atomicAdd(&P.counts[b], (unsigned long long)s);
    }
    W.since_flush = 0;
}

// One span of neighbour points [j0, j1). The home point (hx, hy, hz) is
// already moved into the neighbour grid's frame for this span. If masked,
// only neighbours with index > the lane's home index count (autocorrelation
// inside the home tile).
// Queue the ambiguous pairs of one neighbour point for the FP64 re-test.
template <int MODE, int EST>
__device__ __forceinline__ void enqueue(const CountArgs& P, WaveState& W, const float2* B1,
                                        const float2* B2, const double* T1, const double* T2,
                                        int lane, bool amb, uint32_t hidx, uint32_t j, float hx,
                                        float hy, float hz, float hlx, float hly, float hlz,
                                        const float4& q) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(amb);
    if (m == 0) return;
    const float dx = hx - q.x, dy = hy - q.y, dz = hz - q.z;
    float lx = 0.f, ly = 0.f, lz = 0.f;
    if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
        lx = hlx + q.x;
        ly = hly + q.y;
        lz = hlz + q.z;
    }
    uint32_t tent;
    (void)classify32<MODE, EST, true>(P, B1, B2, dx, dy, dz, lx, ly, lz, &tent);
    const uint32_t pre =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (amb) {
        const uint32_t pos = W.tail + pre;
        W.qi[pos] = hidx;
        W.qj[pos] = j;
        W.qt[pos] = tent;
    }
    W.tail += (uint32_t)__popcll(m);
    if (W.tail >= 64u) drain_queue<MODE, EST>(P, W, T1, T2, lane, false);
}

// U neighbour points per step: their scalar loads are issued together and
// the U classifications form one straight-line block that the compiler can
// interleave; the LDS increments and the (rare) re-test queueing follow.
template <int MODE, int PREC, int EST, bool MASKED, uint32_t U>
__device__ __forceinline__ void step32(const CountArgs& P, WaveState& W, const float2* B1,
                                       const float2* B2, const double* T1, const double* T2,
                                       int lane, bool valid, uint32_t hidx, float hx, float hy,
                                       float hz, float hlx, float hly, float hlz, uint32_t j) {
    float4 q[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) q[u] = load_u32x4f(P.B.p32, j + u);
    uint32_t bin[U];
    bool cnt[U], amb[U];
#pragma unroll
    for (uint32_t u = 0; u < U; u++) {
        const bool act = valid & (!MASKED | (j + u > hidx));
        const float dx = hx - q[u].x, dy = hy - q[u].y, dz = hz - q[u].z;
        float lx = 0.f, ly = 0.f, lz = 0.f;
        if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
            lx = hlx + q[u].x;
            ly = hly + q[u].y;
            lz = hlz + q[u].z;
        }
        if (PREC == P_FP32O) {
            uint32_t tent;
            (void)classify32<MODE, EST, true>(P, B1, B2, dx, dy, dz, lx, ly, lz, &tent);
            cnt[u] = act && tent != kNoBin;
            bin[u] = tent;
            amb[u] = false;
        } else {
            const C32 c = classify32<MODE, EST, false>(P, B1, B2, dx, dy, dz, lx, ly, lz, nullptr);
            cnt[u] = act & c.in;
            amb[u] = act & !(c.in | c.out);
            bin[u] = c.bin;
        }
    }
    // the wave-wide "any ambiguous" vote is taken before the increments so
    // that the ambiguity masks are consumed while they are still compare results
    uint64_t any_amb = 0;
    if (PREC == P_FP32E) {
        bool any = false;
#pragma unroll
        for (uint32_t u = 0; u < U; u++) any = any | amb[u];
        any_amb = __builtin_amdgcn_ballot_w64(any);
    }
#pragma unroll
    for (uint32_t u = 0; u < U; u++)
        if (cnt[u]) hist_add(W.hist, bin[u], P.copies, lane);
    if (PREC == P_FP32E) {
        if (any_amb) {
#pragma unroll
            for (uint32_t u = 0; u < U; u++)
                enqueue<MODE, EST>(P, W, B1, B2, T1, T2, lane, amb[u], hidx, j + u, hx, hy, hz,
                                   hlx, hly, hlz, q[u]);
        }
    }
}

template <int MODE, int PREC, int EST, bool MASKED>
__device__ void run_span32(const CountArgs& P, WaveState& W, const float2* B1, const float2* B2,
                           const double* T1, const double* T2, int lane, bool valid,
                           uint32_t hidx, float hx, float hy, float hz, float hlx, float hly,
                           float hlz, uint32_t j0, uint32_t j1) {
    constexpr uint32_t U = 4;
    uint32_t j = j0;
    for (; j + U <= j1; j += U)
        step32<MODE, PREC, EST, MASKED, U>(P, W, B1, B2, T1, T2, lane, valid, hidx, hx, hy, hz,
                                           hlx, hly, hlz, j);
    for (; j < j1; j++)
        step32<MODE, PREC, EST, MASKED, 1>(P, W, B1, B2, T1, T2, lane, valid, hidx, hx, hy, hz,
                                           hlx, hly, hlz, j);
}

template <int MODE, int EST, bool MASKED>
__device__ void run_span64(const CountArgs& P, WaveState& W, const double* T1, const double* T2,
                           int lane, bool valid, uint32_t hidx, double hx, double hy, double hz,
                           double sx, double sy, double sz, uint32_t j0, uint32_t j1) {
    const bool shifted = (sx != 0.0) || (sy != 0.0) || (sz != 0.0);
    for (uint32_t j = j0; j < j1; j++) {
        const P64 q = load_u64x3(P.B.p64, j);
        bool act = valid && (!MASKED || j > hidx);
        double dx = hx - q.x, dy = hy - q.y, dz = hz - q.z;
        if (shifted) {
            // the span's periodic image: the same result as the minimum-image
            // wrap for every pair the stencil can pair up (see host notes)
            dx = dx - sx;
            dy = dy - sy;
            dz = dz - sz;
        }
        double lx = 0.0, ly = 0.0, lz = 0.0;
        if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
            lx = hx + q.x;
            ly = hy + q.y;
            lz = hz + q.z;
        }
        int k1 = 0, k2 = 0;
        double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
        float v = (float)d2;
        if (MODE == M_MONO || MODE == M_THETA) {
            k1 = guess1<MODE, EST>(P, v);
        } else if (MODE == M_RMU_Z) {
            k1 = guess1<M_MONO, EST>(P, v);
            float rinv = __builtin_amdgcn_rsqf(v);
            k2 = guess_lin(fabsf((float)dz) * rinv, P.e2a, P.e2b, P.n2m1);
        } else if (MODE == M_RMU_MID) {
            k1 = guess1<M_MONO, EST>(P, v);
            float sl = (float)fma(dz, lz, fma(dy, ly, dx * lx));
            float ll = (float)fma(lz, lz, fma(ly, ly, lx * lx));
            float mu = fabsf(sl) * __builtin_amdgcn_rsqf(v * ll);
            k2 = guess_lin(mu, P.e2a, P.e2b, P.n2m1);
        } else {
            float sl = (float)fma(dz, lz, fma(dy, ly, dx * lx));
            float ll = (float)fma(lz, lz, fma(ly, ly, lx * lx));
            float rll = __builtin_amdgcn_rcpf(ll);
            float pi2 = sl * sl * rll;
            float sg2 = fmaxf(v - pi2, 0.0f);
            k1 = guess_lin(__builtin_amdgcn_sqrtf(sg2), P.e1a, P.e1b, P.n1m1);
            k2 = guess_lin(__builtin_amdgcn_sqrtf(pi2), P.e2a, P.e2b, P.n2m1);
        }
        uint32_t k = classify64<MODE>(P, T1, T2, dx, dy, dz, lx, ly, lz, k1, k2);
        if (act && k != kNoBin) hist_add(W.hist, k, P.copies, lane);
    }
}

// Process one span (possibly split into a masked head inside the home tile
// and an unmasked rest), in chunks that keep the LDS counters below 2^32.
template <int MODE, int PREC, int EST>
__device__ void do_span(const CountArgs& P, WaveState& W, const float2* B1, const float2* B2,
                        const double* T1, const double* T2, int lane, bool valid, uint32_t hidx,
                        uint32_t nhome, uint32_t ts, uint32_t te, bool same, float hx32,
                        float hy32, float hz32, double hx64, double hy64, double hz64, double sx,
                        double sy, double sz, uint32_t j0, uint32_t j1) {
    if (j1 <= j0) return;
    // FP32 home point in this span's frame, and the midpoint helper hx + lc
    float ex = hx32 - (float)sx, ey = hy32 - (float)sy, ez = hz32 - (float)sz;
    float elx = 0.f, ely = 0.f, elz = 0.f;
    if (MODE == M_RMU_MID || MODE == M_SIGMAPI) {
        elx = ex + P.lcx;
        ely = ey + P.lcy;
        elz = ez + P.lcz;
    }
    uint32_t a = j0;
    if (same) {
        // neighbours inside the home tile: only j > i; before the tile: none
        uint32_t m0 = ts + 1u > j0 ? ts + 1u : j0;
        uint32_t m1 = te < j1 ? te : j1;
        if (m1 > m0) {
            // lanes 0..(j - ts - 1) pair with neighbour j: sum of (j - ts) over the head
            const uint64_t lo_ = m0 - ts, hi_ = m1 - 1u - ts;
            const uint64_t pairs = (lo_ + hi_) * (hi_ - lo_ + 1u) / 2u;
            if (W.since_flush + pairs >= 0xfffffff0ull) wave_flush<MODE, EST>(P, W, T1, T2, lane);
            W.since_flush += pairs;
            W.evals += pairs;
            if (PREC == P_FP64)
                run_span64<MODE, EST, true>(P, W, T1, T2, lane, valid, hidx, hx64, hy64, hz64, sx,
                                            sy, sz, m0, m1);
            else
                run_span32<MODE, PREC, EST, true>(P, W, B1, B2, T1, T2, lane, valid, hidx, ex, ey,
                                                  ez, elx, ely, elz, m0, m1);
        }
        a = te > j0 ? te : j0;
    }
    while (a < j1) {
        uint32_t b = (j1 - a > kChunk) ? a + kChunk : j1;
        uint64_t pairs = (uint64_t)nhome * (uint64_t)(b - a);
        if (W.since_flush + pairs >= 0xfffffff0ull) wave_flush<MODE, EST>(P, W, T1, T2, lane);
        W.since_flush += pairs;
        W.evals += pairs;
        if (PREC == P_FP64)
            run_span64<MODE, EST, false>(P, W, T1, T2, lane, valid, hidx, hx64, hy64, hz64, sx, sy,
                                         sz, a, b);
        else
            run_span32<MODE, PREC, EST, false>(P, W, B1, B2, T1, T2, lane, valid, hidx, ex, ey, ez,
                                               elx, ely, elz, a, b);
        a = b;
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ int imod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Enumerate the neighbour spans of one home tile and count them.
template <int MODE, int PREC, int EST>
__device__ void do_tile(const CountArgs& P, WaveState& W, const float2* B1, const float2* B2,
                        const double* T1, const double* T2, int lane, const Tile& tl) {
    const uint32_t ts = tl.start, te = tl.end;
    const uint32_t nhome = te - ts;
    const int c0 = (int)(tl.c0c1 & 0xffffu), c1 = (int)(tl.c0c1 >> 16);
    const GridView& A = P.A;
    const GridView& B = P.B;
    const int cy = (int)(tl.row % (uint32_t)A.ny), cz = (int)(tl.row / (uint32_t)A.ny);
    const bool valid = (uint32_t)lane < nhome;
    const uint32_t hidx = ts + (uint32_t)lane;
    float hx32 = 0.f, hy32 = 0.f, hz32 = 0.f;
    double hx64 = 0.0, hy64 = 0.0, hz64 = 0.0;
    if (valid) {
        if (PREC == P_FP64) {
            P64 p = A.p64[hidx];
            hx64 = p.x;
            hy64 = p.y;
            hz64 = p.z;
        } else {
            float4 p = A.p32[hidx];
            hx32 = p.x + P.offx;
            hy32 = p.y + P.offy;
            hz32 = p.z + P.offz;
        }
    }
    W.tiles++;
    const double R = P.Rs;

    if (P.geom == CUTE_GEOM_SPHERE) {
        // tile pixel block: phi in [c0, c1+1) * ax, cos theta in one band
        const double zlo = A.oy + cy * A.ay, zhi = zlo + A.ay;
        const double zl = fmax(-1.0, fmin(1.0, zlo)), zh = fmax(-1.0, fmin(1.0, zhi));
        const double th_lo = acos(zh), th_hi = acos(zl);
        const double ts_ = P.th_s;
        const double zn_hi = (th_lo - ts_ <= 0.0) ? 1.0 : cos(th_lo - ts_);
        const double zn_lo = (th_hi + ts_ >= kPi) ? -1.0 : cos(th_hi + ts_);
        int b0 = (int)floor((zn_lo - B.oy) / B.ay) - 1, b1 = (int)floor((zn_hi - B.oy) / B.ay) + 1;
        b0 = clampi(b0, 0, B.ny - 1);
        b1 = clampi(b1, 0, B.ny - 1);
        // half-width in phi of a cap of radius th_s around any tile point:
        // asin(sin th_s / sin theta) at the tile colatitude nearest a pole
        const double zmax2 = fmax(zl * zl, zh * zh);
        const double smin = sqrt(fmax(0.0, 1.0 - zmax2));
        bool full = !(P.sin_th_s < smin * (1.0 - 1e-9)) || (P.th_s >= 0.5 * kPi);
        double hw = full ? 0.0 : asin(P.sin_th_s / smin) * (1.0 + 1e-9) + 1e-12;
        const double phlo = c0 * A.ax - hw, phhi = (c1 + 1) * A.ax + hw;
        int x0 = (int)floor(phlo / B.ax) - 1, x1 = (int)floor(phhi / B.ax) + 1;
        if (x1 - x0 + 1 >= B.nx) full = true;
        for (int by = b0; by <= b1; by++) {
            const int byu = unii(by);
            const bool same = P.is_auto && byu == cy;
            if (P.is_auto && byu < cy) continue;
            const uint32_t rb = (uint32_t)byu * (uint32_t)B.nx;
            int pa[2][2];
            int np = 0;
            if (same) {
                // index rule inside the home band: partners with larger index,
                // i.e. cells >= c0 up to the right reach, plus the left reach
                // that wraps past phi = 2 pi onto the band's last cells
                if (full) {
                    pa[np][0] = c0;
                    pa[np][1] = B.nx - 1;
                    np++;
                } else {
                    int r1 = x1 < B.nx - 1 ? x1 : B.nx - 1;
                    int s2 = x0 < 0 ? x0 + B.nx : B.nx;  // start of wrapped left part
                    if (s2 <= r1 + 1) {
                        pa[np][0] = c0;
                        pa[np][1] = B.nx - 1;
                        np++;
                    } else {
                        pa[np][0] = c0;
                        pa[np][1] = r1;
                        np++;
                        if (s2 <= B.nx - 1) {
                            pa[np][0] = s2;
                            pa[np][1] = B.nx - 1;
                            np++;
                        }
                    }
                }
            } else if (full) {
                pa[0][0] = 0;
                pa[0][1] = B.nx - 1;
                np = 1;
            } else {
                // cyclic range [x0, x1] (length < nx) split at the phi wrap
                int a0 = imod(x0, B.nx);
                int len = x1 - x0 + 1;
                if (a0 + len <= B.nx) {
                    pa[0][0] = a0;
                    pa[0][1] = a0 + len - 1;
                    np = 1;
                } else {
                    pa[0][0] = a0;
                    pa[0][1] = B.nx - 1;
                    pa[1][0] = 0;
                    pa[1][1] = a0 + len - 1 - B.nx;
                    np = 2;
                }
            }
            for (int q = 0; q < np; q++) {
                const cu32p cs = (cu32p)(const void*)B.cstart;
                uint32_t j0 = uni(cs[rb + (uint32_t)pa[q][0]]);
                uint32_t j1 = uni(cs[rb + (uint32_t)pa[q][1] + 1u]);
                const bool chk = same && pa[q][0] == c0;
                do_span<MODE, PREC, EST>(P, W, B1, B2, T1, T2, lane, valid, hidx, nhome, ts, te,
                                         chk, hx32, hy32, hz32, hx64, hy64, hz64, 0.0, 0.0, 0.0, j0,
                                         j1);
            }
        }
        return;
    }

    // 3-D boxes: the tile box, grown by R, selects rows of neighbour cells
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
    const double R2 = R * R;
    for (int bz = z0; bz <= z1; bz++) {
        for (int by = y0; by <= y1; by++) {
            const int bzu = unii(bz), byu = unii(by);
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
            double sy = 0.0, sz = 0.0;
            int ry = byu, rz = bzu;
            if (P.periodic) {
                const int ky = floordiv(byu, B.ny), kz = floordiv(bzu, B.nz);
                ry = byu - ky * B.ny;
                rz = bzu - kz * B.nz;
                sy = ky * P.L;
                sz = kz * P.L;
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
                const int u0 = a0 - kx * B.nx, u1 = a1 - kx * B.nx;
                const cu32p cs = (cu32p)(const void*)B.cstart;
                uint32_t j0 = uni(cs[rb + (uint32_t)u0]);
                uint32_t j1 = uni(cs[rb + (uint32_t)u1 + 1u]);
                const double sx = kx * P.L;
                const bool chk = same && kx == 0 && a0 == c0;
                do_span<MODE, PREC, EST>(P, W, B1, B2, T1, T2, lane, valid, hidx, nhome, ts, te,
                                         chk, hx32, hy32, hz32, hx64, hy64, hz64, sx, sy, sz, j0,
                                         j1);
                a0 = a1 + 1;
            }
        }
    }
}

template <int MODE, int PREC, int EST>
__global__ __launch_bounds__(256) void k_count(CountArgs P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int n1 = P.n1, n2 = P.n2;
    const int n2p = n2 > 0 ? n2 : 0;
    double* T1 = reinterpret_cast<double*>(smem);
    double* T2 = T1 + (n1 + 1);
    float2* B1 = reinterpret_cast<float2*>(T2 + (n2p + 1));
    float2* B2 = B1 + n1;
    uint32_t* hist0 = reinterpret_cast<uint32_t*>(B2 + (n2p > 0 ? n2p : 1));
    uint32_t* q0 = hist0 + (size_t)nwaves * P.hist_words;
    for (int i = threadIdx.x; i <= n1; i += blockDim.x) T1[i] = P.T1[i];
    for (int i = threadIdx.x; i <= n2p; i += blockDim.x) T2[i] = n2p ? P.T2[i] : 0.0;
    if (PREC != P_FP64) {
        for (int i = threadIdx.x; i < n1; i += blockDim.x) B1[i] = P.band1[i];
        for (int i = threadIdx.x; i < n2p; i += blockDim.x) B2[i] = P.band2[i];
    }
    for (int i = threadIdx.x; i < nwaves * P.hist_words; i += blockDim.x) hist0[i] = 0u;
    __syncthreads();

    WaveState W;
    W.hist = hist0 + (size_t)wave * P.hist_words;
    W.qi = q0 + (size_t)wave * 3 * kQCap;
    W.qj = W.qi + kQCap;
    W.qt = W.qj + kQCap;
    W.tail = 0;
    W.since_flush = 0;
    W.evals = W.retests = W.flips = W.tiles = 0;

    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(P.work_head, 1u);
        t = uni(t);
        if (t >= P.ntiles) break;
        const cu32p tp = (cu32p)(const void*)P.tiles;
        Tile tl;
        tl.start = uni(tp[4 * t]);
        tl.end = uni(tp[4 * t + 1]);
        tl.row = uni(tp[4 * t + 2]);
        tl.c0c1 = uni(tp[4 * t + 3]);
        do_tile<MODE, PREC, EST>(P, W, B1, B2, T1, T2, lane, tl);
    }
    if (PREC == P_FP32E) drain_queue<MODE, EST>(P, W, T1, T2, lane, true);
    if (lane == 0) {
        atomicAdd(&P.stats[0], (unsigned long long)W.evals);
        atomicAdd(&P.stats[1], (unsigned long long)W.retests);
        atomicAdd(&P.stats[2], (unsigned long long)W.flips);
        atomicAdd(&P.stats[3], (unsigned long long)W.tiles);
    }
    __syncthreads();
    // sum the waves' histograms and their copies, then one atomic per bin
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) {
        uint64_t s = 0;
        for (int w = 0; w < nwaves; w++) {
            const uint32_t* h = hist0 + (size_t)w * P.hist_words + (size_t)b * P.copies;
            for (int c = 0; c < P.copies; c++) s += h[c];
        }
        if (s) atomicAdd(&P.counts[b], (unsigned long long)s);
    }
}

template <int MODE, int PREC, int EST>
cute_status launch_one(const CountArgs& a, int wg_waves, size_t lds, hipStream_t s, int* grid_used) {
    auto kern = k_count<MODE, PREC, EST>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_status(e, "hipFuncSetAttribute");
    }
    int dev = 0, ncu = 0, per_cu = 0;
    CUTE_HIP(hipGetDevice(&dev));
    CUTE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    CUTE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wg_waves, lds));
    if (per_cu < 1) per_cu = 1;
    int64_t want = (int64_t)per_cu * ncu;
    int64_t need = ((int64_t)a.ntiles + wg_waves - 1) / wg_waves;
    int grid = (int)(want < need ? want : need);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * wg_waves), lds, s, a);
    CUTE_HIP(hipGetLastError());
    if (grid_used) *grid_used = grid;
    return CUTE_OK;
}

template <int MODE, int PREC>
cute_status launch_est(const CountArgs& a, int est, int wg_waves, size_t lds, hipStream_t s,
                       int* g) {
    if (est == E_LOG) return launch_one<MODE, PREC, E_LOG>(a, wg_waves, lds, s, g);
    return launch_one<MODE, PREC, E_LIN>(a, wg_waves, lds, s, g);
}

template <int MODE>
cute_status launch_prec(const CountArgs& a, int prec, int est, int wg_waves, size_t lds,
                        hipStream_t s, int* g) {
    switch (prec) {
        case P_FP64: return launch_est<MODE, P_FP64>(a, est, wg_waves, lds, s, g);
        case P_FP32E: return launch_est<MODE, P_FP32E>(a, est, wg_waves, lds, s, g);
        default: return launch_est<MODE, P_FP32O>(a, est, wg_waves, lds, s, g);
    }
}

}  // namespace

cute_status launch_count(const CountArgs& args, int mode, int prec, int est, int wg_waves,
                         size_t lds_bytes, hipStream_t stream, int* grid_used) {
    switch (mode) {
        case M_MONO: return launch_prec<M_MONO>(args, prec, est, wg_waves, lds_bytes, stream, grid_used);
        case M_RMU_Z: return launch_prec<M_RMU_Z>(args, prec, est, wg_waves, lds_bytes, stream, grid_used);
        case M_RMU_MID: return launch_prec<M_RMU_MID>(args, prec, est, wg_waves, lds_bytes, stream, grid_used);
        case M_SIGMAPI: return launch_prec<M_SIGMAPI>(args, prec, est, wg_waves, lds_bytes, stream, grid_used);
        case M_THETA: return launch_prec<M_THETA>(args, prec, est, wg_waves, lds_bytes, stream, grid_used);
        default: return fail(CUTE_E_INTERNAL, "unknown mode");
    }
}

// Home tiles: each row of cells is cut into runs of at most 64 points whose
// x-extent stays within max_w cells (so that periodic stencils never wrap
// onto themselves). One thread walks one row.
__global__ __launch_bounds__(256) void k_tiles_count(const uint32_t* __restrict__ cstart, int nx,
                                                     int nrows, int max_w, uint32_t* __restrict__ ntile) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t* cs = cstart + (size_t)r * nx;
    uint32_t cnt = 0, fill = 0;
    int first = -1;
    for (int c = 0; c < nx; c++) {
        uint32_t left = cs[c + 1] - cs[c];
        while (left > 0) {
            if (fill == 0 || fill == 64u || c - first + 1 > max_w) {
                cnt++;
                fill = 0;
                first = c;
            }
            uint32_t take = 64u - fill < left ? 64u - fill : left;
            fill += take;
            left -= take;
        }
    }
    ntile[r] = cnt;
}

__global__ __launch_bounds__(256) void k_tiles_write(const uint32_t* __restrict__ cstart, int nx,
                                                     int nrows, int max_w,
                                                     const uint32_t* __restrict__ toff,
                                                     Tile* __restrict__ tiles) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t* cs = cstart + (size_t)r * nx;
    uint32_t o = toff[r];
    uint32_t fill = 0;
    int first = -1;
    Tile cur;
    bool open = false;
    for (int c = 0; c < nx; c++) {
        uint32_t pos = cs[c];
        uint32_t left = cs[c + 1] - cs[c];
        while (left > 0) {
            if (!open || fill == 64u || c - first + 1 > max_w) {
                if (open) tiles[o++] = cur;
                open = true;
                fill = 0;
                first = c;
                cur.start = pos;
                cur.end = pos;
                cur.row = (uint32_t)r;
                cur.c0c1 = (uint32_t)c | ((uint32_t)c << 16);
            }
            uint32_t take = 64u - fill < left ? 64u - fill : left;
            fill += take;
            left -= take;
            pos += take;
            cur.end = pos;
            cur.c0c1 = (cur.c0c1 & 0xffffu) | ((uint32_t)c << 16);
        }
    }
    if (open) tiles[o++] = cur;
}

cute_status build_tiles(const GridHost& g, int max_w, hipStream_t s, Tile** tiles,
                        uint32_t* ntiles) {
    *tiles = nullptr;
    *ntiles = 0;
    const int nrows = g.ny * g.nz;
    TempList tmp(s);
    uint32_t* cnt = nullptr;
    cute_status st = tmp.alloc(&cnt, (size_t)nrows + 1);
    if (st != CUTE_OK) return st;
    const unsigned nb = (unsigned)((nrows + 255) / 256);
    hipLaunchKernelGGL(k_tiles_count, dim3(nb), dim3(256), 0, s, g.cstart, g.nx, nrows, max_w, cnt);
    CUTE_HIP(hipGetLastError());
    CUTE_HIP(hipMemsetAsync(cnt + nrows, 0, sizeof(uint32_t), s));
    if ((st = exclusive_scan(cnt, cnt, (size_t)nrows + 1, s)) != CUTE_OK) return st;
    uint32_t total = 0;
    CUTE_HIP(hipMemcpyAsync(&total, cnt + nrows, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CUTE_HIP(hipStreamSynchronize(s));
    Tile* t = nullptr;
    if ((st = dalloc(&t, total, s)) != CUTE_OK) return st;
    if (total > 0) {
        hipLaunchKernelGGL(k_tiles_write, dim3(nb), dim3(256), 0, s, g.cstart, g.nx, nrows, max_w,
                           cnt, t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            dfree(t, s);
            return hip_status(e, "tiles launch");
        }
    }
    *tiles = t;
    *ntiles = total;
    return CUTE_OK;
}

}  // namespace cute
