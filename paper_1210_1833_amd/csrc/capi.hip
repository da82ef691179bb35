// Host side of the C ABI: argument validation, decision thresholds and their
// FP32 rounding bands, launch planning, and the estimators.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "cute_internal.h"
#include "runtime.h"

namespace cute {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

cute_status fail(cute_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

cute_status hip_status(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(CUTE_E_OUT_OF_MEMORY, m);
    return fail(CUTE_E_DEVICE, m);
}

cute_status ensure_device_ready(int* device) {
    static std::mutex mu;
    static bool ready[64] = {false};
    int dev = 0;
    CUTE_HIP(hipGetDevice(&dev));
    *device = dev;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && !ready[dev]) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        ready[dev] = true;
    }
    return CUTE_OK;
}

namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr float kBig = 1e30f;
constexpr int kQCap = 128;                        // must match the kernels
constexpr int kSpanCap = 192;                     // must match the kernels

float up32(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}
float dn32(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}

bool edges_ok(const double* e, int n, bool mu) {
    if (!e || n < 1) return false;
    for (int k = 0; k <= n; k++) {
        if (!std::isfinite(e[k]) || e[k] < 0.0) return false;
        if (mu && e[k] > 1.0) return false;
        if (k > 0 && !(e[k] > e[k - 1])) return false;
    }
    return true;
}

bool is_linear(const double* e, int n) {
    const double s = (e[n] - e[0]) / n;
    for (int k = 0; k <= n; k++)
        if (std::fabs(e[k] - (e[0] + k * s)) > 1e-6 * s) return false;
    return true;
}

bool is_log(const double* e, int n) {
    if (!(e[0] > 0.0)) return false;
    const double a = std::log2(e[0]), s = (std::log2(e[n]) - a) / n;
    for (int k = 0; k <= n; k++)
        if (std::fabs(std::log2(e[k]) - (a + k * s)) > 1e-6 * s) return false;
    return true;
}

// Bound on |FP32 squared separation - exact r^2| plus |canonical FP64 value -
// exact r^2| for a true separation up to r. FP32 components carry absolute
// errors <= ec (coordinate rounding, origin shift, subtraction); the three-term
// sum of squares adds <= 3.01 u of itself. The FP64 canonical value has the
// same structure with ec64 and u64.
double d2_bound(double r, double ec, double ec64) {
    const double s3 = std::sqrt(3.0);
    const double d32 = 2 * s3 * r * ec + 3 * ec * ec + 3.01 * kU32 * (r + s3 * ec) * (r + s3 * ec);
    const double d64 =
        2 * s3 * r * ec64 + 3 * ec64 * ec64 + 3.01 * kU64 * (r + s3 * ec64) * (r + s3 * ec64);
    return d32 + d64;
}

struct Plan {
    int mode = 0, est = 0;
    double rmax = 0.0;               // largest countable separation
    std::vector<double> T1, T2;      // canonical thresholds
    std::vector<float2> band1, band2;
    CountArgs a;
};

cute_status make_thresholds(const cute_binning* b, Plan& pl) {
    const int n1 = b->n1, n2 = b->n2;
    pl.T1.resize(n1 + 1);
    for (int k = 0; k <= n1; k++) {
        if (b->kind == CUTE_BIN_THETA) {
            const double c = 2.0 * std::sin(0.5 * b->edges1[k]);  // chord of theta_k
            pl.T1[k] = c * c;
        } else {
            pl.T1[k] = b->edges1[k] * b->edges1[k];
        }
    }
    if (n2 > 0) {
        pl.T2.resize(n2 + 1);
        for (int k = 0; k <= n2; k++) pl.T2[k] = b->edges2[k] * b->edges2[k];
    } else {
        pl.T2.assign(1, 0.0);
    }
    if (b->kind == CUTE_BIN_SIGMAPI)
        pl.rmax = std::sqrt(b->edges1[n1] * b->edges1[n1] + b->edges2[n2] * b->edges2[n2]);
    else if (b->kind == CUTE_BIN_THETA)
        pl.rmax = 2.0 * std::sin(0.5 * b->edges1[n1]);
    else
        pl.rmax = b->edges1[n1];
    return CUTE_OK;
}

}  // namespace
}  // namespace cute

using namespace cute;

extern "C" const char* cute_status_string(cute_status s) {
    switch (s) {
        case CUTE_OK: return "ok";
        case CUTE_E_INVALID_ARG: return "invalid argument";
        case CUTE_E_UNSUPPORTED: return "unsupported";
        case CUTE_E_OUT_OF_MEMORY: return "out of memory";
        case CUTE_E_DEVICE: return "device error";
        case CUTE_E_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

extern "C" const char* cute_last_error(void) { return g_err.c_str(); }

static cute_status validate_binning(const cute_binning* b) {
    if (!b) return fail(CUTE_E_INVALID_ARG, "binning is NULL");
    if (b->kind < CUTE_BIN_MONO || b->kind > CUTE_BIN_THETA)
        return fail(CUTE_E_INVALID_ARG, "unknown bin kind");
    if (b->n1 < 1 || b->n1 > 65536) return fail(CUTE_E_INVALID_ARG, "n1 must be in [1, 65536]");
    if (!edges_ok(b->edges1, b->n1, false))
        return fail(CUTE_E_INVALID_ARG, "edges1 must be finite, >= 0 and strictly increasing");
    if (b->kind == CUTE_BIN_THETA && b->edges1[b->n1] > 3.14159265358979323846)
        return fail(CUTE_E_INVALID_ARG, "theta edges must be <= pi");
    if (b->kind == CUTE_BIN_RMU || b->kind == CUTE_BIN_SIGMAPI) {
        if (b->n2 < 1 || b->n2 > 65536) return fail(CUTE_E_INVALID_ARG, "n2 must be in [1, 65536]");
        if (!edges_ok(b->edges2, b->n2, b->kind == CUTE_BIN_RMU))
            return fail(CUTE_E_INVALID_ARG,
                        "edges2 must be finite, >= 0, strictly increasing (mu within [0, 1])");
        if (b->los != CUTE_LOS_Z && b->los != CUTE_LOS_MIDPOINT)
            return fail(CUTE_E_INVALID_ARG, "unknown line of sight");
        if (b->kind == CUTE_BIN_SIGMAPI && b->los != CUTE_LOS_MIDPOINT)
            return fail(CUTE_E_UNSUPPORTED, "sigma-pi needs the midpoint line of sight");
        if ((int64_t)b->n1 * b->n2 > (int64_t)1 << 24)
            return fail(CUTE_E_INVALID_ARG, "too many bins");
    } else if (b->n2 != 0) {
        return fail(CUTE_E_INVALID_ARG, "n2 must be 0 for MONO and THETA");
    }
    return CUTE_OK;
}

extern "C" cute_status cute_count_pairs(const cute_grid* ga, const cute_grid* gb,
                                        const cute_binning* bins, cute_precision prec,
                                        uint64_t* counts, int32_t counts_on_device,
                                        cute_count_stats* st, void* stream) {
    if (!ga) return fail(CUTE_E_INVALID_ARG, "grid a is NULL");
    if (!counts) return fail(CUTE_E_INVALID_ARG, "counts is NULL");
    cute_status s = validate_binning(bins);
    if (s != CUTE_OK) return s;
    if (prec != CUTE_PREC_FP64 && prec != CUTE_PREC_FP32_EDGE && prec != CUTE_PREC_FP32_ONLY)
        return fail(CUTE_E_INVALID_ARG, "unknown precision");
    const bool is_auto = (gb == nullptr || gb == ga);
    if (!gb) gb = ga;
    const GridHost& A = ga->h;
    const GridHost& B = gb->h;
    if (A.geom != B.geom) return fail(CUTE_E_INVALID_ARG, "grids have different geometries");
    const bool sphere = A.geom == CUTE_GEOM_SPHERE;
    const bool periodic = A.geom == CUTE_GEOM_BOX_PERIODIC;
    if (sphere != (bins->kind == CUTE_BIN_THETA))
        return fail(CUTE_E_INVALID_ARG, "THETA binning needs SPHERE grids and vice versa");
    if (periodic && A.L != B.L) return fail(CUTE_E_INVALID_ARG, "periodic grids with different L");
    const bool mid = (bins->kind == CUTE_BIN_SIGMAPI) ||
                     (bins->kind == CUTE_BIN_RMU && bins->los == CUTE_LOS_MIDPOINT);
    if (mid && periodic)
        return fail(CUTE_E_UNSUPPORTED, "midpoint line of sight in a periodic box");

    int dev = 0;
    if ((s = ensure_device_ready(&dev)) != CUTE_OK) return s;
    hipStream_t hs = (hipStream_t)stream;

    Plan pl;
    make_thresholds(bins, pl);
    const int n1 = bins->n1, n2 = bins->n2 > 0 ? bins->n2 : 0;
    const int nbins = n1 * (n2 > 0 ? n2 : 1);
    const double rmax = pl.rmax;
    if (periodic && !(rmax * (1.0 + 1e-9) < 0.5 * A.L))
        return fail(CUTE_E_INVALID_ARG, "periodic r_max must be < L/2");

    switch (bins->kind) {
        case CUTE_BIN_MONO: pl.mode = M_MONO; break;
        case CUTE_BIN_THETA: pl.mode = M_THETA; break;
        case CUTE_BIN_RMU: pl.mode = bins->los == CUTE_LOS_Z ? M_RMU_Z : M_RMU_MID; break;
        default: pl.mode = M_SIGMAPI; break;
    }

    CountArgs& a = pl.a;
    memset(&a, 0, sizeof(a));
    a.A = A.view();
    a.B = B.view();
    a.geom = (int)A.geom;
    a.is_auto = is_auto ? 1 : 0;
    a.periodic = periodic ? 1 : 0;
    a.L = periodic ? A.L : 0.0;
    a.n1 = n1;
    a.n2 = n2;
    a.nbins = nbins;
    a.n1m1 = (float)(n1 - 1);
    a.n2m1 = (float)(n2 > 0 ? n2 - 1 : 0);
    a.mu_top_closed = (bins->kind == CUTE_BIN_RMU && bins->edges2[n2] >= 1.0) ? 1 : 0;

    // ---- stencil radius ----------------------------------------------------
    const double scale = std::max({A.ext, B.ext, 1e-300});
    a.Rs = rmax * (1.0 + 1e-9) + 1e-9 * scale;
    if (sphere) {
        const double th = bins->edges1[n1];
        a.th_s = th * (1.0 + 1e-9) + 1e-12;
        a.sin_th_s = std::sin(std::min(a.th_s, 0.5 * 3.14159265358979323846));
    }

    // ---- home-tile width limit ---------------------------------------------
    int max_w;
    if (periodic) {
        // a tile plus its reach must not wrap onto itself in any axis
        const double reach_y = (A.ay + 2 * a.Rs) / B.ay + 2.0;
        const double reach_z = (A.az + 2 * a.Rs) / B.az + 2.0;
        if (reach_y > B.ny || reach_z > B.nz)
            return fail(CUTE_E_INVALID_ARG,
                        "periodic grid too coarse for this r_max (build it with r_max set)");
        const double w = ((B.nx - 2) * B.ax - 2 * a.Rs) / A.ax;
        max_w = (int)std::floor(w);
        if (max_w < 1)
            return fail(CUTE_E_INVALID_ARG,
                        "periodic grid too coarse for this r_max (build it with r_max set)");
        max_w = std::min(max_w, std::max(1, (int)std::floor(0.5 * a.Rs / A.ax)));
    } else if (sphere) {
        max_w = std::max(1, (int)std::floor(0.5 * a.th_s / A.ax));
    } else {
        max_w = std::max(1, (int)std::floor(0.5 * a.Rs / A.ax));
    }
    max_w = std::min(max_w, 65535);

    // ---- FP32 error model --------------------------------------------------
    // ec bounds |FP32 coordinate difference - exact difference| per component:
    // rounding of both FP32 copies (u X_A + u X_B), the neighbour moved into
    // the home frame, q - off with off = FP32(cA - cB) or a periodic image
    // shift (u |off| + u (X_B + |off|)), and the final subtraction (u R).
    double offmax = 0.0;
    if (periodic) {
        offmax = A.L;
    } else if (!sphere && !is_auto) {
        offmax = std::max({std::fabs((double)(float)(A.cx - B.cx)),
                           std::fabs((double)(float)(A.cy - B.cy)),
                           std::fabs((double)(float)(A.cz - B.cz))});
    }
    a.offx = is_auto || periodic || sphere ? 0.f : (float)(A.cx - B.cx);
    a.offy = is_auto || periodic || sphere ? 0.f : (float)(A.cy - B.cy);
    a.offz = is_auto || periodic || sphere ? 0.f : (float)(A.cz - B.cz);
    const double Re = rmax * 1.01 + 1e-30;
    const double extra = offmax > 0.0 ? kU32 * offmax + kU32 * (B.ext + offmax) : 0.0;
    const double ec = 1.0001 * (kU32 * A.ext + kU32 * B.ext + extra + kU32 * Re);
    const double ec64 = 2.0 * kU64 * (A.rawmax + B.rawmax + (periodic ? A.L : 0.0)) * 1.0001;
    const double s3 = std::sqrt(3.0);

    // ---- dimension-1 estimate and bands ------------------------------------
    const double* e1 = bins->edges1;
    const bool lin1 = is_linear(e1, n1), log1 = !lin1 && is_log(e1, n1);
    pl.est = log1 ? E_LOG : E_LIN;
    if (bins->kind == CUTE_BIN_SIGMAPI) pl.est = E_LIN;  // sigma estimated linearly
    {
        const double lo = e1[0], hi = e1[n1];
        if (pl.est == E_LOG) {
            const double la = std::log2(lo), ls = (std::log2(hi) - la) / n1;
            if (bins->kind == CUTE_BIN_THETA) {
                a.e1a = (float)(1.0 / ls);          // t = log2(theta)
                a.e1b = (float)(-la / ls);
            } else {
                a.e1a = (float)(0.5 / ls);          // t = log2(r^2)
                a.e1b = (float)(-la / ls);
            }
        } else {
            const double sp = (hi - lo) / n1;
            a.e1a = (float)(1.0 / sp);
            a.e1b = (float)(-lo / sp);
        }
    }
    if (n2 > 0) {
        const double lo = bins->edges2[0], hi = bins->edges2[n2];
        const double sp = (hi - lo) / n2;
        a.e2a = (float)(1.0 / sp);
        a.e2b = (float)(-lo / sp);
        a.d2_generic = is_linear(bins->edges2, n2) ? 0 : 1;
    }

    if (bins->kind == CUTE_BIN_SIGMAPI) {
        pl.band1.resize(n1);
        for (int k = 0; k < n1; k++) {
            float lo = pl.T1[k] == 0.0 ? kBig : -(float)pl.T1[k];
            float hi = -(float)pl.T1[k + 1];
            pl.band1[k] = make_float2(lo, hi);
        }
        a.out_hi = -(float)pl.T1[n1];
        a.out_lo = pl.T1[0] == 0.0 ? kBig : -(float)pl.T1[0];
    } else {
        std::vector<float> lo_e(n1 + 1), hi_e(n1 + 1);
        for (int k = 0; k <= n1; k++) {
            const double rk = std::sqrt(pl.T1[k]);
            const double m = 1.5 * d2_bound(rk * (1.0 + 1e-6) + 2.0 * ec, ec, ec64);
            lo_e[k] = pl.T1[k] == 0.0 ? -1.0f : up32(pl.T1[k] + m);
            const double h = pl.T1[k] - m;
            hi_e[k] = h > 0.0 ? dn32(h) : -1.0f;
        }
        pl.band1.resize(n1);
        for (int k = 0; k < n1; k++) pl.band1[k] = make_float2(lo_e[k], hi_e[k + 1]);
        a.out_hi = lo_e[n1];
        a.out_lo = hi_e[0];
    }
    a.bot32 = (float)pl.T1[0];
    a.top32 = (float)pl.T1[n1];

    // ---- dimension-2 (mu or pi) tables and ratio-predicate bands -------------
    if (n2 > 0) {
        pl.band2.resize(n2);
        for (int k = 0; k < n2; k++) {
            float lo = pl.T2[k] == 0.0 ? kBig : -(float)pl.T2[k];
            float hi = (k + 1 == n2 && a.mu_top_closed) ? -kBig : -(float)pl.T2[k + 1];
            pl.band2[k] = make_float2(lo, hi);
        }
        a.nlo2_first = pl.T2[0] == 0.0 ? kBig : -(float)pl.T2[0];
        a.nhi2_last = a.mu_top_closed ? -kBig : -(float)pl.T2[n2];
        a.d2lo32 = (float)pl.T2[0];
        a.d2hi32 = (float)pl.T2[n2];
        if (bins->kind == CUTE_BIN_RMU) a.d2_partial = (pl.T2[0] > 0.0 || !a.mu_top_closed) ? 1 : 0;
    } else {
        pl.band2.assign(1, make_float2(0.f, 0.f));
    }
    if (pl.mode == M_RMU_Z) {
        // |F - exact| <= 2 sqrt(2) ec r + 3 ec^2 + 8.1 u S, plus the FP64 terms;
        // r is bounded by the FP32 estimate r (1 + 5u) + sqrt(3) ec
        const double k1 = 2 * std::sqrt(2.0) * ec + (2 + 2 * s3) * ec64;
        // the kernel uses delta = dA0 + dA1 r with the v term folded in:
        // A2 v <= A2 Re r for every pair whose mu decision counts (r < Re)
        const double a2 = 1.5 * (8.1 * kU32 + 16 * kU64) * 1.0001;
        a.dA1 = (float)((1.5 * k1 * (1 + 8 * kU32) + a2 * Re) * 1.0001);
        a.dA0 = (float)(1.5 * (k1 * s3 * ec + 3 * ec * ec + 4 * ec64 * ec64) * 1.0001);
        a.dA2 = 0.0f;
    } else if (mid) {
        // midpoint line of sight: perturbations of s = p - q (per component
        // <= ec) and l = p + q (per component <= el) move the ratio predicates
        // by first-order terms ~ r |s-error| ll and r^2 |l| |l-error|
        // l = h + ((q - off) + FP32(2 cA)): the roundings of both copies, of the
        // frame shift, of 2 cA, of the two additions (|l| <= max|p| + max|q|)
        const double ca = std::max({std::fabs(A.cx), std::fabs(A.cy), std::fabs(A.cz)});
        const double el = 1.0001 * kU32 *
                          (A.ext + B.ext + extra + 2 * ca + (B.ext + offmax + 2 * ca) +
                           (A.lmax + B.lmax));
        const double es = s3 * ec, esl = s3 * el;
        const double es64 = s3 * ec64, el64 = s3 * 2.0 * kU64 * (A.lmax + B.lmax);
        auto fill = [&](double c_lin, double c_round, double kmax2, float* A0, float* A1, float* A2,
                        float* B0, float* B1, float* B2, float* C2, float* C0) {
            // c_lin: multiplier of the first-order terms (4 for mu and sigma, 2 for pi)
            double a1 = c_lin * (es + es64);
            double a2 = c_round * (kU32 + kU64);
            double a0 = 5 * (kU32 + kU64) * kmax2 + 6 * es * es + a1 * s3 * ec + a2 * 3 * ec * ec;
            double b2 = c_lin * (esl + el64) + 2 * esl * a2;
            double b1 = 2 * esl * a1 + c_lin * esl * 3.47 * ec + 4 * es * esl;
            double b0 = 2 * (esl + el64) * kmax2 + 2 * esl * a0 + c_lin * esl * 3 * ec * ec;
            double c2 = 12 * esl * esl + esl * esl * a2;
            double c0 = 2 * kmax2 * esl * esl + esl * esl * a0;
            const double f = 2.0;
            *A0 = (float)(f * a0);
            *A1 = (float)(f * a1);
            *A2 = (float)(f * a2);
            *B0 = (float)(f * b0);
            *B1 = (float)(f * b1);
            *B2 = (float)(f * b2);
            *C2 = (float)(f * c2);
            *C0 = (float)(f * c0);
        };
        if (bins->kind == CUTE_BIN_SIGMAPI) {
            const double smax2 = pl.T1[n1], pmax2 = pl.T2[n2];
            fill(4.0, 15.5, smax2, &a.sA0, &a.sA1, &a.sA2, &a.sB0, &a.sB1, &a.sB2, &a.sC2, &a.sC0);
            fill(2.0, 8.2, pmax2, &a.dA0, &a.dA1, &a.dA2, &a.dB0, &a.dB1, &a.dB2, &a.dC2, &a.dC0);
        } else {
            fill(4.0, 17.5, 1.0, &a.dA0, &a.dA1, &a.dA2, &a.dB0, &a.dB1, &a.dB2, &a.dC2, &a.dC0);
        }
        a.lcx = (float)(2.0 * A.cx);
        a.lcy = (float)(2.0 * A.cy);
        a.lcz = (float)(2.0 * A.cz);
    }

    // ---- LDS plan: one shared 64-bit histogram per 4-wave workgroup --------
    // About 40 KB per workgroup keeps four workgroups (16 waves) on a CU; the
    // copies of the histogram are cut to fit, then the budget is relaxed for
    // very large histograms (fewer workgroups per CU).
    const size_t tables = 8 * (size_t)(n1 + 1) + 8 * (size_t)(n2 + 1) + 8 * (size_t)n1 +
                          8 * (size_t)std::max(n2, 1);
    const int W = 4;
    const size_t per_wave = 12 * (size_t)kQCap + 16 + 12 * (size_t)kSpanCap;
    const size_t fixed = tables + (size_t)W * per_wave;
    int C = 0;
    for (size_t budget : {(size_t)40 * 1024, (size_t)80 * 1024, (size_t)160 * 1024}) {
        if (fixed + 8 * (size_t)nbins > budget) continue;
        size_t cmax = (budget - fixed) / (8 * (size_t)nbins);
        C = 1;
        while (C * 2 <= (int)std::min<size_t>(cmax, 32)) C *= 2;
        break;
    }
    if (C == 0) return fail(CUTE_E_UNSUPPORTED, "histogram does not fit in LDS");
    a.copies = C;
    a.hist_words = nbins * C;
    const size_t lds = fixed + 8 * (size_t)a.hist_words;

    // ---- device buffers ----------------------------------------------------
    TempList tmp(hs);
    double *dT1, *dT2;
    float2 *dB1, *dB2;
    unsigned long long* work;  // counts[nbins], stats[4], head
    CountArgs* dargs;
    if ((s = tmp.alloc(&dT1, pl.T1.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dT2, pl.T2.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dB1, pl.band1.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dB2, pl.band2.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&work, (size_t)nbins + 5)) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dargs, 1)) != CUTE_OK) return s;
    CUTE_HIP(hipMemcpyAsync(dT1, pl.T1.data(), pl.T1.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dT2, pl.T2.data(), pl.T2.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dB1, pl.band1.data(), pl.band1.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dB2, pl.band2.data(), pl.band2.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemsetAsync(work, 0, ((size_t)nbins + 5) * 8, hs));
    a.T1 = dT1;
    a.T2 = dT2;
    a.band1 = dB1;
    a.band2 = dB2;
    a.counts = work;
    a.stats = work + nbins;
    a.work_head = reinterpret_cast<uint32_t*>(work + nbins + 4);

    Tile* tiles = nullptr;
    uint32_t ntiles = 0;
    if (A.n > 0 && B.n > 0) {
        if ((s = build_tiles(A, max_w, hs, &tiles, &ntiles)) != CUTE_OK) return s;
    }
    a.tiles = tiles;
    a.ntiles = ntiles;
    a.self = dargs;
    CUTE_HIP(hipMemcpyAsync(dargs, &a, sizeof(a), hipMemcpyHostToDevice, hs));

    double ms = 0.0;
    int grid = 0;
    if (ntiles > 0) {
        EventTimer timer(hs);
        s = launch_count(a, pl.mode, (int)prec, pl.est, W, lds, hs, &grid);
        if (s != CUTE_OK) {
            dfree(tiles, hs);
            return s;
        }
        ms = timer.stop_ms();
    }
    dfree(tiles, hs);

    if (counts_on_device) {
        CUTE_HIP(hipMemcpyAsync(counts, work, (size_t)nbins * 8, hipMemcpyDeviceToDevice, hs));
    } else {
        CUTE_HIP(hipMemcpyAsync(counts, work, (size_t)nbins * 8, hipMemcpyDeviceToHost, hs));
    }
    unsigned long long hst[4] = {0, 0, 0, 0};
    CUTE_HIP(hipMemcpyAsync(hst, work + nbins, sizeof(hst), hipMemcpyDeviceToHost, hs));
    CUTE_HIP(hipStreamSynchronize(hs));
    if (st) {
        st->pair_evals = hst[0];
        st->retests = hst[1];
        st->flips = hst[2];
        st->tiles = hst[3];
        st->ms_count = ms;
        uint64_t tot = 0;
        if (!counts_on_device)
            for (int k = 0; k < nbins; k++) tot += counts[k];
        st->pairs_in_range = counts_on_device ? 0 : tot;
    }
    if (hst[3] != ntiles) return fail(CUTE_E_INTERNAL, "not every tile was processed");
    return CUTE_OK;
}

// ---------------------------------------------------------------------------
// Estimators (Sec. 2.2) and multipoles (Sec. 2.1), host only.
// ---------------------------------------------------------------------------
// __int128 -> double through the compiler's correctly rounded conversion
static double i128_to_double(__int128 v) { return static_cast<double>(v); }

extern "C" cute_status cute_xi_estimate(cute_estimator e, const uint64_t* dd, const uint64_t* dr,
                                        const uint64_t* rr, int64_t nd, int64_t nr,
                                        const cute_binning* bins, double box_size, double* xi) {
    cute_status s = validate_binning(bins);
    if (s != CUTE_OK) return s;
    if (!dd || !xi) return fail(CUTE_E_INVALID_ARG, "NULL counts or output");
    const int nbins = bins->n1 * (bins->n2 > 0 ? bins->n2 : 1);
    if (e == CUTE_EST_BOX) {
        if (bins->kind != CUTE_BIN_MONO) return fail(CUTE_E_INVALID_ARG, "BOX needs a MONO binning");
        if (!(box_size > 0.0) || !std::isfinite(box_size))
            return fail(CUTE_E_INVALID_ARG, "BOX needs box_size > 0");
        if (nd < 2) return fail(CUTE_E_INVALID_ARG, "nd must be >= 2");
        const double vol = box_size * box_size * box_size;
        const double npairs = 0.5 * (double)nd * (double)(nd - 1);
        const double pi = 3.14159265358979323846;
        for (int k = 0; k < nbins; k++) {
            const double lo = bins->edges1[k], hi = bins->edges1[k + 1];
            const double shell = (4.0 / 3.0) * pi * (hi * hi * hi - lo * lo * lo);
            const double expect = npairs * (shell / vol);
            xi[k] = expect > 0.0 ? (double)dd[k] / expect - 1.0 : NAN;
        }
        return CUTE_OK;
    }
    if (e != CUTE_EST_NATURAL && e != CUTE_EST_LS) return fail(CUTE_E_INVALID_ARG, "unknown estimator");
    if (!rr) return fail(CUTE_E_INVALID_ARG, "rr is NULL");
    if (e == CUTE_EST_LS && !dr) return fail(CUTE_E_INVALID_ARG, "dr is NULL");
    if (nd < 2 || nr < 2) return fail(CUTE_E_INVALID_ARG, "nd and nr must be >= 2");
    if (nd > ((int64_t)1 << 40) || nr > ((int64_t)1 << 40))
        return fail(CUTE_E_INVALID_ARG, "catalog sizes too large for exact arithmetic");
    const __int128 cdd = (__int128)nr * (nr - 1);   // multiplies DD
    const __int128 cdr = (__int128)(nr - 1) * (nd - 1);
    const __int128 crr = (__int128)nd * (nd - 1);   // multiplies RR (and the denominator)
    for (int k = 0; k < nbins; k++) {
        if (rr[k] == 0) {
            xi[k] = NAN;
            continue;
        }
        if (dd[k] > ((uint64_t)1 << 62) || rr[k] > ((uint64_t)1 << 62) ||
            (dr && dr[k] > ((uint64_t)1 << 62)))
            return fail(CUTE_E_INVALID_ARG, "counts too large for exact arithmetic");
        __int128 num, den = crr * (__int128)rr[k];
        if (e == CUTE_EST_NATURAL)
            num = cdd * (__int128)dd[k] - crr * (__int128)rr[k];
        else
            num = cdd * (__int128)dd[k] - cdr * (__int128)dr[k] + crr * (__int128)rr[k];
        xi[k] = i128_to_double(num) / i128_to_double(den);
    }
    return CUTE_OK;
}

// Legendre P_l(x) by the three-term recursion.
static double legendre(int l, double x) {
    if (l == 0) return 1.0;
    double p0 = 1.0, p1 = x;
    for (int n = 1; n < l; n++) {
        const double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

extern "C" cute_status cute_xi_multipoles(const double* xi_rmu, const cute_binning* bins,
                                          int32_t n_ell, const int32_t* ells, double* out) {
    cute_status s = validate_binning(bins);
    if (s != CUTE_OK) return s;
    if (bins->kind != CUTE_BIN_RMU) return fail(CUTE_E_INVALID_ARG, "multipoles need an RMU binning");
    if (!xi_rmu || !ells || !out || n_ell < 1) return fail(CUTE_E_INVALID_ARG, "NULL or empty argument");
    for (int a = 0; a < n_ell; a++)
        if (ells[a] < 0 || ells[a] % 2 || ells[a] > 64)
            return fail(CUTE_E_INVALID_ARG, "ells must be even, in [0, 64]");
    const int n1 = bins->n1, n2 = bins->n2;
    const double* m = bins->edges2;
    for (int a = 0; a < n_ell; a++) {
        const int l = ells[a];
        // (2l+1) int_{m_j}^{m_{j+1}} P_l = [P_{l+1} - P_{l-1}] evaluated at the ends
        std::vector<double> w(n2);
        for (int j = 0; j < n2; j++) {
            if (l == 0)
                w[j] = m[j + 1] - m[j];
            else
                w[j] = (legendre(l + 1, m[j + 1]) - legendre(l - 1, m[j + 1])) -
                       (legendre(l + 1, m[j]) - legendre(l - 1, m[j]));
        }
        for (int i = 0; i < n1; i++) {
            double acc = 0.0;
            for (int j = 0; j < n2; j++) acc += xi_rmu[(size_t)i * n2 + j] * w[j];
            out[(size_t)a * n1 + i] = acc;
        }
    }
    return CUTE_OK;
}
