// Launch planning shared by the single and the batched counts: decision
// thresholds of a binning, per-pair geometry of two grids, the proven FP32
// rounding bands and the LDS layout of a count kernel. Host code only.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "cute_internal.h"
#include "runtime.h"

namespace cute {

namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr float kBig = 1e30f;
constexpr double kPiH = 3.14159265358979323846;
constexpr uint32_t kBiasBits = 0x4B000000u;       // bits of the float 2^23
// largest relative error assumed of the hardware 1/sqrt (v_rsq_f32); it is
// documented at 1 ulp (2^-23), so this keeps a factor 4
constexpr double kRsqRel = 0x1p-21;

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

}  // namespace

cute_status validate_binning(const cute_binning* b) {
    if (!b) return fail(CUTE_E_INVALID_ARG, "binning is NULL");
    if (b->kind < CUTE_BIN_MONO || b->kind > CUTE_BIN_THETA)
        return fail(CUTE_E_INVALID_ARG, "unknown bin kind");
    if (b->n1 < 1 || b->n1 > 65536) return fail(CUTE_E_INVALID_ARG, "n1 must be in [1, 65536]");
    if (!edges_ok(b->edges1, b->n1, false))
        return fail(CUTE_E_INVALID_ARG, "edges1 must be finite, >= 0 and strictly increasing");
    if (b->kind == CUTE_BIN_THETA && b->edges1[b->n1] > kPiH)
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

bool same_binning(const cute_binning* a, const cute_binning* b) {
    if (a == b) return true;
    if (a->kind != b->kind || a->n1 != b->n1 || a->n2 != b->n2) return false;
    if ((a->kind == CUTE_BIN_RMU || a->kind == CUTE_BIN_SIGMAPI) && a->los != b->los) return false;
    if (memcmp(a->edges1, b->edges1, sizeof(double) * (size_t)(a->n1 + 1)) != 0) return false;
    if (a->n2 > 0 && memcmp(a->edges2, b->edges2, sizeof(double) * (size_t)(a->n2 + 1)) != 0)
        return false;
    return true;
}

// Thresholds and the bin-estimate constants of a validated binning.
void plan_binning(const cute_binning* b, Plan& pl) {
    const int n1 = b->n1, n2 = b->n2 > 0 ? b->n2 : 0;
    CountArgs& a = pl.a;
    memset(&a, 0, sizeof(a));
    switch (b->kind) {
        case CUTE_BIN_MONO: pl.mode = M_MONO; break;
        case CUTE_BIN_THETA: pl.mode = M_THETA; break;
        case CUTE_BIN_RMU: pl.mode = b->los == CUTE_LOS_Z ? M_RMU_Z : M_RMU_MID; break;
        default: pl.mode = M_SIGMAPI; break;
    }
    // canonical thresholds: squared edges (chords of theta)
    pl.T1.resize(n1 + 1);
    for (int k = 0; k <= n1; k++) {
        if (b->kind == CUTE_BIN_THETA) {
            const double c = 2.0 * std::sin(0.5 * b->edges1[k]);
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

    a.n1 = n1;
    a.n2 = n2;
    a.nbins = n1 * (n2 > 0 ? n2 : 1);
    a.n1m1 = (float)(n1 - 1);
    a.n2m1 = (float)(n2 > 0 ? n2 - 1 : 0);
    a.mu_top_closed = (b->kind == CUTE_BIN_RMU && b->edges2[n2] >= 1.0) ? 1 : 0;

    // dimension-1 estimate
    const double* e1 = b->edges1;
    const bool lin1 = is_linear(e1, n1), log1 = !lin1 && is_log(e1, n1);
    pl.est = log1 ? E_LOG : E_LIN;
    if (b->kind == CUTE_BIN_SIGMAPI) pl.est = E_LIN;  // sigma estimated linearly
    {
        const double lo = e1[0], hi = e1[n1];
        if (pl.est == E_LOG) {
            const double la = std::log2(lo), ls = (std::log2(hi) - la) / n1;
            if (b->kind == CUTE_BIN_THETA) {
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
    a.bot32 = (float)pl.T1[0];
    a.top32 = (float)pl.T1[n1];
    a.top64 = pl.T1[n1];
    if (b->kind == CUTE_BIN_SIGMAPI) {
        // sigma^2 + pi^2 = r^2 exactly for the FP64 differences and any line
        // of sight; the canonical products err by a few ulp of r^2 |l|^2, far
        // inside a 1e-12 relative margin
        const double r2 = b->edges1[n1] * b->edges1[n1] + b->edges2[n2] * b->edges2[n2];
        a.top64 = std::nextafter(r2 * (1.0 + 1e-12), INFINITY);
    }
    // biased FP32 estimates: fma(t + s, a, 2^23) rounds to 2^23 + floor(t a + b)
    // when s = (b - 1/2) / a; the clamps are the bits of 2^23 + n - 1
    a.n2p1 = n2 > 0 ? n2 : 1;
    a.s1 = (float)(((double)a.e1b - 0.5) / (double)a.e1a);
    a.top1 = kBiasBits + (uint32_t)(n1 - 1);
    a.top2 = kBiasBits + (uint32_t)(a.n2p1 - 1);

    // dimension 2 (mu or pi): estimate and the ratio-predicate tables
    if (n2 > 0) {
        const double lo = b->edges2[0], hi = b->edges2[n2];
        const double sp = (hi - lo) / n2;
        a.e2a = (float)(1.0 / sp);
        a.e2b = (float)(-lo / sp);
        a.d2_generic = is_linear(b->edges2, n2) ? 0 : 1;
        a.s2 = (float)(((double)a.e2b - 0.5) / (double)a.e2a);
        pl.band2.resize(n2);
        for (int k = 0; k < n2; k++) {
            float l = pl.T2[k] == 0.0 ? kBig : -(float)pl.T2[k];
            float h = (k + 1 == n2 && a.mu_top_closed) ? -kBig : -(float)pl.T2[k + 1];
            pl.band2[k] = make_float2(l, h);
        }
        a.nlo2_first = pl.T2[0] == 0.0 ? kBig : -(float)pl.T2[0];
        a.nhi2_last = a.mu_top_closed ? -kBig : -(float)pl.T2[n2];
        a.d2lo32 = (float)pl.T2[0];
        a.d2hi32 = (float)pl.T2[n2];
        if (b->kind == CUTE_BIN_RMU) a.d2_partial = (pl.T2[0] > 0.0 || !a.mu_top_closed) ? 1 : 0;
    } else {
        pl.band2.assign(1, make_float2(0.f, 0.f));
    }
}

// Geometry of one pair of grids under a binning: compatibility checks, the
// stencil radius, the home-tile width limit, the FP32 frame offsets and the
// inputs of the rounding-error model.
cute_status plan_item(const GridHost& A, const GridHost& B, bool is_auto, const cute_binning* b,
                      const Plan& pl, ItemGeom* g) {
    if (A.geom != B.geom) return fail(CUTE_E_INVALID_ARG, "grids have different geometries");
    const bool sphere = A.geom == CUTE_GEOM_SPHERE;
    const bool periodic = A.geom == CUTE_GEOM_BOX_PERIODIC;
    if (sphere != (b->kind == CUTE_BIN_THETA))
        return fail(CUTE_E_INVALID_ARG, "THETA binning needs SPHERE grids and vice versa");
    if (periodic && A.L != B.L) return fail(CUTE_E_INVALID_ARG, "periodic grids with different L");
    const bool mid = (b->kind == CUTE_BIN_SIGMAPI) ||
                     (b->kind == CUTE_BIN_RMU && b->los == CUTE_LOS_MIDPOINT);
    if (mid && periodic) return fail(CUTE_E_UNSUPPORTED, "midpoint line of sight in a periodic box");
    const double rmax = pl.rmax;
    if (periodic && !(rmax * (1.0 + 1e-9) < 0.5 * A.L))
        return fail(CUTE_E_INVALID_ARG, "periodic r_max must be < L/2");

    *g = ItemGeom();
    g->A = A.view();
    g->B = B.view();
    g->geom = (int)A.geom;
    g->is_auto = is_auto ? 1 : 0;
    g->periodic = periodic ? 1 : 0;
    g->L = periodic ? A.L : 0.0;

    // stencil radius
    const double scale = std::max({A.ext, B.ext, 1e-300});
    g->Rs = rmax * (1.0 + 1e-9) + 1e-9 * scale;
    if (sphere) {
        const double th = b->edges1[b->n1];
        g->th_s = th * (1.0 + 1e-9) + 1e-12;
        g->sin_th_s = std::sin(std::min(g->th_s, 0.5 * kPiH));
    }

    // home-tile width limit
    int max_w;
    if (periodic) {
        // a tile plus its reach must not wrap onto itself in any axis
        const double reach_y = (A.ay + 2 * g->Rs) / B.ay + 2.0;
        const double reach_z = (A.az + 2 * g->Rs) / B.az + 2.0;
        if (reach_y > B.ny || reach_z > B.nz)
            return fail(CUTE_E_INVALID_ARG,
                        "periodic grid too coarse for this r_max (build it with r_max set)");
        const double w = ((B.nx - 2) * B.ax - 2 * g->Rs) / A.ax;
        max_w = (int)std::floor(w);
        if (max_w < 1)
            return fail(CUTE_E_INVALID_ARG,
                        "periodic grid too coarse for this r_max (build it with r_max set)");
        max_w = std::min(max_w, std::max(1, (int)std::floor(0.5 * g->Rs / A.ax)));
    } else if (sphere) {
        max_w = std::max(1, (int)std::floor(0.5 * g->th_s / A.ax));
    } else {
        max_w = std::max(1, (int)std::floor(0.5 * g->Rs / A.ax + 0.5));
    }
    g->max_w = std::min(max_w, 65535);

    // FP32 error model. ec bounds |FP32 coordinate difference - exact
    // difference| per component: rounding of both FP32 copies (u X_A + u X_B),
    // the neighbour moved into the home frame, q - off with off = FP32(cA - cB)
    // or a periodic image shift (u |off| + u (X_B + |off|)), and the final
    // subtraction (u R).
    double offmax = 0.0;
    if (periodic) {
        offmax = A.L;
    } else if (!sphere && !is_auto) {
        offmax = std::max({std::fabs((double)(float)(A.cx - B.cx)),
                           std::fabs((double)(float)(A.cy - B.cy)),
                           std::fabs((double)(float)(A.cz - B.cz))});
    }
    const bool no_off = is_auto || periodic || sphere;
    g->offx = no_off ? 0.f : (float)(A.cx - B.cx);
    g->offy = no_off ? 0.f : (float)(A.cy - B.cy);
    g->offz = no_off ? 0.f : (float)(A.cz - B.cz);
    const double Re = rmax * 1.01 + 1e-30;
    const double extra = offmax > 0.0 ? kU32 * offmax + kU32 * (B.ext + offmax) : 0.0;
    g->em.ec = 1.0001 * (kU32 * A.ext + kU32 * B.ext + extra + kU32 * Re);
    g->em.ec64 = 2.0 * kU64 * (A.rawmax + B.rawmax + (periodic ? A.L : 0.0)) * 1.0001;
    if (mid) {
        // l = h + ((q - off) + FP32(2 cA)): the roundings of both copies, of the
        // frame shift, of 2 cA, of the two additions (|l| <= max|p| + max|q|)
        const double ca = std::max({std::fabs(A.cx), std::fabs(A.cy), std::fabs(A.cz)});
        g->em.el = 1.0001 * kU32 *
                   (A.ext + B.ext + extra + 2 * ca + (B.ext + offmax + 2 * ca) + (A.lmax + B.lmax));
        g->em.el64 = 2.0 * kU64 * (A.lmax + B.lmax);
        g->lcx = (float)(2.0 * A.cx);
        g->lcy = (float)(2.0 * A.cy);
        g->lcz = (float)(2.0 * A.cz);
    }

    // Neighbour rows as offsets, when both grids have one geometry (always
    // for an autocorrelation): the gap between the home row and the row at
    // offset (dy, dz) is (|dy| - 1) a_y by (|dz| - 1) a_z, and the cells
    // within R of the tile's x-range [c0, c1] are c0 - ceil(w / a_x) ..
    // c1 + 1 + floor(w / a_x) with w^2 = R^2 - gap^2. Rounded outward, so the
    // rows and cells are a superset of those the exact distances select.
    const bool same_geom = !sphere && A.nx == B.nx && A.ny == B.ny && A.nz == B.nz &&
                           A.ox == B.ox && A.oy == B.oy && A.oz == B.oz && A.ax == B.ax &&
                           A.ay == B.ay && A.az == B.az;
    if (same_geom) {
        const double R = g->Rs * (1.0 + 1e-12);
        const int ry = (int)std::ceil(R / A.ay) + 1, rz = (int)std::ceil(R / A.az) + 1;
        for (int dz = -rz; dz <= rz; dz++)
            for (int dy = -ry; dy <= ry; dy++) {
                if (is_auto && (dz < 0 || (dz == 0 && dy < 0))) continue;
                const double gy = std::max(0, std::abs(dy) - 1) * A.ay;
                const double gz = std::max(0, std::abs(dz) - 1) * A.az;
                const double rem = R * R - gy * gy - gz * gz;
                if (rem <= 0.0) continue;
                const double wc = std::sqrt(rem) / A.ax * (1.0 + 1e-12) + 1e-9;
                const int left = (int)std::ceil(wc), right = (int)std::floor(wc) + 1;
                g->stencil.push_back(make_int4(dy, dz, left, right));
            }
        // nearest rows first: a chunk that spans the end of one row and the
        // start of the next then holds neighbours at similar distances, so
        // that whole steps past the top edge are more common
        auto gap2 = [&](const int4& e) {
            const double gy = std::max(0, std::abs(e.x) - 1) * A.ay;
            const double gz = std::max(0, std::abs(e.y) - 1) * A.az;
            return gy * gy + gz * gz;
        };
        std::stable_sort(g->stencil.begin(), g->stencil.end(),
                         [&](const int4& u, const int4& v) { return gap2(u) < gap2(v); });
        if (g->stencil.size() > 65536) g->stencil.clear();
    }

    // estimated candidate pairs: nA nB times the stencil's share of B's domain
    double vol_b, vol_s;
    if (sphere) {
        vol_b = std::max(B.nx * B.ax * B.ny * B.ay, 1e-300);  // phi range x cos(theta) range
        vol_s = kPiH * g->th_s * g->th_s;
    } else {
        vol_b = std::max(B.nx * B.ax * B.ny * B.ay * B.nz * B.az, 1e-300);
        vol_s = 4.0 / 3.0 * kPiH * g->Rs * g->Rs * g->Rs;
    }
    g->cost = (double)A.n * (double)B.n * std::min(1.0, 1.5 * vol_s / vol_b) * (is_auto ? 0.5 : 1.0);
    return CUTE_OK;
}

// The error model of several items: every term of the bounds grows with each
// input, so the component-wise maximum bounds every item.
ErrModel max_err(const ErrModel& x, const ErrModel& y) {
    ErrModel m;
    m.ec = std::max(x.ec, y.ec);
    m.ec64 = std::max(x.ec64, y.ec64);
    m.el = std::max(x.el, y.el);
    m.el64 = std::max(x.el64, y.el64);
    return m;
}

// Rounding bands of the midpoint line of sight (sigma, pi and mu against the
// pair midpoint, Sec. 2.1 with l = p + q). Every constant below is a term of
// the bound derived in the design notes; the FP32 operation order it assumes
// is the one of classify32. Notation: s = p - q and l = p + q of the FP64
// inputs (exact reals); the FP32 vectors carry |s32 - s| <= es and
// |l32 - l| <= fe (norms); x is sigma or pi, T an edge's squared value;
// Rv bounds |s| for every pair the FP32 path decides (v32 < skip32); the
// direction error of l is phi = fe / |l| <= 1/15 once ll >= llg.
//   |x32^2 - x^2| <= 2 x Dx + Dx^2,  Dx = es + 2 r phi   (x32 of the FP32 inputs)
// (x = |s.n| or |s x n| with n = l / |l|, and |n32 - n| <= 2 phi). Split into
// a per-edge part that multiplies ll and goes into the band tables,
//   b(T) = M [2 x' es + es^2 + E64 + cu u Rv^2 + 6 u T],  x' = sqrt(T + E64),
// with cu the rounding of the FP32 products (14 for sigma: |s|^2 |l|^2 -
// (s.l)^2 with both terms rounded; 8 for pi: (s.l)^2) and 6 u T the rounding
// of ll, of the threshold product and of the final fma, and a per-pair part
// in the units of F (t = K1 |l| + K0) for the terms in phi:
//   ll (4 (x + es) r phi + 4 r^2 phi^2) <= K1 |l32| + K0.
// E64 bounds the canonical FP64 decision's own deviation from exact reals.
static void midpoint_bands(const cute_binning* b, const ErrModel& em, Plan& pl) {
    CountArgs& a = pl.a;
    const int n1 = b->n1, n2 = b->n2;
    const double s3 = std::sqrt(3.0), u = kU32;
    const double es = s3 * em.ec;            // |s32 - s|
    const double fe = s3 * em.el;            // |l32 - l|
    const double kg = 16.0;                  // guard: |l32| >= kg fe
    const double ig = 1.0 / (1.0 - 1.0 / kg);
    const double lrel = 1.0 + 2.0 * kRsqRel; // |l32| <= fl(ll rsq(ll)) (1 + 2^-20)
    const double M = 1.25;                   // safety factor on the derived bound
    a.llg = up32(kg * kg * fe * fe * (1.0 + 4 * u));
    if (pl.mode == M_SIGMAPI) {
        // |s| of any pair with v32 < skip32 (skip32 covers the FP32 and FP64
        // errors of d2 up to there)
        const double Rv = std::sqrt((double)a.skip32 * (1.0 + 3.02 * u)) + es;
        const double Tmax = std::max(pl.T1[n1], pl.T2[n2]);
        const double E64 = 64.0 * kU64 * (Rv * Rv + Tmax);
        const double xmax = std::sqrt(Tmax + E64) * (1.0 + 1e-9);
        a.spK1 = up32((1.0 + 4 * u) * 4.0 * (xmax + es) * Rv * fe * lrel * ig);
        a.spK0 = up32((1.0 + 4 * u) * 4.0 * Rv * Rv * fe * fe * ig * ig + 1e-30);
        auto band = [&](double T, double cu) {
            const double x = std::sqrt(T + E64) * (1.0 + 1e-9);
            return M * (2 * x * es + es * es + E64 + cu * u * Rv * Rv + 6 * u * T + 1e-30) /
                   (1.0 - 6 * u);
        };
        std::vector<double> bs(n1 + 1), bp(n2 + 1);
        for (int k = 0; k <= n1; k++) bs[k] = band(pl.T1[k], 14.0);
        for (int k = 0; k <= n2; k++) bp[k] = band(pl.T2[k], 8.0);
        // bin k certifies lo <= x^2 - t/ll and x^2 + t/ll <= hi, lo = T_k + b_k
        // and hi = T_{k+1} - b_{k+1}, as |F + m ll| <= H ll - t with m the
        // negated centre and H the half-width of [lo, hi]. A first edge at
        // zero cannot be crossed: the interval is taken as [-hi, hi] (m = 0).
        // With the FP32 m and the two roundings of the kernel's fmas (each at
        // most u of its result), |fl(F + m ll)| <= fl(H ll - t) implies
        // |F - c ll| <= (H (1 + 2.01 u) + |m + c|) ll - t, so H is stored as
        // dn32((Hx - |m + c|) / (1 + 2.01 u)), Hx the exact half-width. A bin
        // with no room (hi <= lo) gets H = -1: never certified.
        auto mid_half = [&](double Tlo, double blo, double Thi, double bhi) {
            const double hi = Thi - bhi;
            const double lo = Tlo == 0.0 ? -hi : Tlo + blo;
            if (!(hi > lo)) return make_float2(0.0f, -1.0f);
            const double c = 0.5 * (lo + hi), hx = 0.5 * (hi - lo);
            const float m = (float)(-c);
            const double h = (hx - std::fabs((double)m + c)) / (1.0 + 2.01 * u);
            return h > 0.0 ? make_float2(m, dn32(h)) : make_float2(0.0f, -1.0f);
        };
        pl.band1.resize(n1);
        for (int k = 0; k < n1; k++)
            pl.band1[k] = mid_half(pl.T1[k], bs[k], pl.T1[k + 1], bs[k + 1]);
        pl.band2.resize(n2);
        for (int k = 0; k < n2; k++)
            pl.band2[k] = mid_half(pl.T2[k], bp[k], pl.T2[k + 1], bp[k + 1]);
        auto hi_w = [](double T, double bb) { return T - bb <= 0.0 ? kBig : up32(-(T - bb)); };
        a.sp_wstop = dn32(-(pl.T1[n1] + bs[n1]));
        a.sp_wptop = dn32(-(pl.T2[n2] + bp[n2]));
        a.sp_wsbot = hi_w(pl.T1[0], bs[0]);
        a.sp_wpbot = hi_w(pl.T2[0], bp[0]);
        a.sp_low = (pl.T1[0] > 0.0 || pl.T2[0] > 0.0) ? 1 : 0;
        return;
    }
    // mu against the midpoint: G = pi^2 - T r^2 (T = mu_j^2 <= 1). With
    // |pi32 - pi| <= es + 2 r phi and |r32^2 - r^2| <= 2 r es + es^2:
    //   |G32 - G| <= 2 r es (mu + T) + es^2 (1 + T) + 4 mu r^2 phi
    //               + 4 r es phi + 4 r^2 phi^2 <= 4 r es + 2 es^2 + 4 r^2 phi + ...
    // and the FP32 evaluation (s.l)^2 - T fl(v ll) errs by at most
    // (6.02 + 1 + 8.04) u r^2 |l|^2. In the kernel's form
    //   delta = ll (A2 v + A1 r + A0) + |l| (B2 v + B1 r + B0) + C2 v + C0,
    // with r the FP32 estimate fl(v rsq(v)) and v = fl(|s32|^2):
    // |s| <= r (1 + 2^-20) + es, |s|^2 <= v (1 + 3.02 u) + 2 r es + es^2.
    const double Rv = pl.rmax * (1.0 + 1e-6) + es;
    const double E64 = 64.0 * kU64 * (Rv * Rv + 1.0);
    const double rr = 1.0 + 2.0 * kRsqRel, vv = (1.0 + 3.02 * u) / (1.0 - 3.02 * u);
    const double A1 = 4 * es * rr;
    const double A2 = 15.1 * u * vv;
    const double A0 = 4 * es * es + 2 * es * es + E64 * (1.0 + 1e-9);
    // l terms: ll phi <= fe |l32| lrel ig, ll phi^2 <= fe^2 ig^2
    const double fl1 = fe * lrel * ig, fl2 = fe * fe * ig * ig;
    const double B2 = 4 * fl1 * vv;                       // 4 r^2 phi ll
    const double B1 = (8 + 4) * fl1 * es * rr;            // 4 (2 r es) + 4 r es (phi ll)
    const double B0 = (4 + 4) * fl1 * es * es;
    const double C2 = 8 * fl2 * vv;                       // 4 r^2 phi^2 ll, r^2 <= 2 v + 2 es^2
    const double C0 = 8 * fl2 * es * es + 1e-30;
    // the kernel's FP32 evaluation of delta (seven roundings of positive
    // terms) and ll against |l32|^2 (3.01 u) lose at most 16 u relative
    const double f = M * (1.0 + 16 * u) / (1.0 - 2 * u);
    a.dA0 = up32(f * A0);
    a.dA1 = up32(f * A1);
    a.dA2 = up32(f * A2);
    a.dB0 = up32(f * B0);
    a.dB1 = up32(f * B1);
    a.dB2 = up32(f * B2);
    a.dC2 = up32(f * C2);
    a.dC0 = up32(f * C0);
}

// The mu decision of the z line of sight in mu space (linear mu edges
// covering [0, 1]). The kernel forms ts2 = fl(|dz32| rsq(v) + s2) and
// x = ts2 a, the pair's position in bin units (bin j is x in [j - 1/2,
// j + 1/2)), and takes its estimated bin j (clamped to the bins) when the
// offset fl(x - j) is at most 1/2 - beta in size.
// With mu = |dz| / r exact, |dz32 - dz| <= ec, |v - r^2| <= D(r) (the d2
// bound) and rsq within kRsqRel:
//   |mu32 - mu| <= (1 + sqrt 3) ec / r + 1.5 ec^2 / r^2 + 1.51 u + kRsqRel
// (mu32 = |dz32| rsq(v) exactly; 1/r <= rsq(v) (1 + kRsqRel) (1 + D / 2 r^2)).
// A pair is certified only when beta < 1/2, i.e. ec / r < 1 / (8 a) here, so
// the second-order terms are below 0.4 % of the first. In bin units,
//   beta = a |mu32 - mu| + a u (1 + |s2|) + u (a + |b| + 1) + a |s2 - s2*|
//          + dev + a E64 + 2 u,
// with s2* the exact shift, dev the largest distance of the caller's edges
// (in bin units) from the integers, E64 = 8 u64 the canonical FP64 mu
// decision's own error, and 2 u for the rounding of the offset and the FP32
// fma of the half-width (the term u (a + |b| + 1) is a margin beyond these
// roundings). Kept as 1/2 - beta =
// muB1 rsq(v) + muB0, times a safety factor 1.5 on beta.
static void mu_space_band(const cute_binning* b, const ErrModel& em, Plan& pl) {
    CountArgs& a = pl.a;
    const int n2 = b->n2;
    const double u = kU32, s3 = std::sqrt(3.0), ec = em.ec;
    const double A = (double)a.e2a, B = (double)a.e2b, S2 = (double)a.s2;
    double dev = 0.0;
    for (int j = 0; j <= n2; j++)
        dev = std::max(dev, std::fabs(b->edges2[j] * A + B - (double)j));
    dev = dev * (1.0 + 1e-9) + 1e-12;
    const double s2x = (B - 0.5) / A;
    const double M = 1.5;
    const double c1 = M * A * ((1.0 + s3) * ec * 1.01 * (1.0 + kRsqRel) + kRsqRel * ec);
    const double c0 = M * (A * (1.51 * u * 1.01 + kRsqRel + u * (1.0 + std::fabs(S2)) * 1.01 +
                                std::fabs(S2 - s2x) + 8.0 * kU64) +
                           u * (A + std::fabs(B) + 1.0) + dev) +
                      2.0 * u;
    a.muB1 = -up32(c1);
    a.muB0 = dn32(0.5 - c0);
    pl.est |= E_MUF;
}

// r in bin units for the z line of sight with linear r bins (Sec. 2.1, r of
// the pair). The kernel forms ts = fl(v rsq(v) + s1) and x = ts a (a, s1 the
// FP32 map: bin k is x in [k - 1/2, k + 1/2)) and certifies the pair inside
// its estimated bin k (clamped to the bins) when |x - k| <= 1/2 - beta; a
// pair outside the bins has |x - k| >= 1/2. At an edge e_k, with ê_k =
// sqrt(T1[k]) (T1[k] the canonical FP64 threshold):
//  - x differs from a (sqrt(v) + s1) by the rsq error a sqrt(v) kRsqRel, the
//    rounding of ts u a (sqrt(v) + |s1|) and the rounding of the offset;
//  - the FP32 map puts the edge at a distance dev_k = |a (ê_k + s1) - (k -
//    1/2)| from ê_k (in x);
//  - a pair with x at least beta past the map's edge has sqrt(v) >= ê_k +
//    delta, delta = (beta - err - dev_k) / a, so v >= T1[k] + 2 ê_k delta;
//    delta >= m_k / (1.5 ê_k) puts v past the v-space band m_k of the edge
//    (the band of the table path), on the side the canonical FP64 compare
//    takes. Below an edge v <= T1[k] - 2 ê_k delta + delta^2, and delta is
//    less than half a bin, at most ê_k / 2 for k >= 1 with e_0 = 0.
// The edge e_0 = 0 cannot be crossed (r >= 0). beta is the largest of these
// terms, times 1.25. Returns false (the count keeps the band tables for r and
// mu) for bins that start above 0 or when beta would leave no room.
static bool r_space_band(const cute_binning* b, const ErrModel& em, Plan& pl) {
    CountArgs& a = pl.a;
    const int n1 = b->n1;
    if (pl.T1[0] != 0.0) return false;
    const double u = kU32, A = (double)a.e1a, S1 = (double)a.s1;
    double beta = 0.0;
    for (int k = 1; k <= n1; k++) {
        const double ek = std::sqrt(pl.T1[k]) * (1.0 + 4.0 * kU64);
        const double m = 1.5 * d2_bound(ek * (1.0 + 1e-6) + 2.0 * em.ec, em.ec, em.ec64) +
                         4.0 * kU64 * pl.T1[k];
        const double rr = ek * 1.01 + 2.0 * em.ec;
        const double err = A * rr * kRsqRel + u * A * (rr + std::fabs(S1)) * 1.01 + 0x1p-24;
        const double dev = std::fabs(A * (ek + S1) - ((double)k - 0.5)) + A * ek * 8.0 * kU64 + 1e-12;
        beta = std::max(beta, err + dev + A * m / (1.5 * ek));
    }
    beta *= 1.25;
    if (!(beta < 0.25)) return false;
    a.rB0 = dn32(0.5 - beta);
    return true;
}

// FP32 rounding bands of the decision thresholds under the error model em.
void plan_bands(const cute_binning* b, const ErrModel& em, Plan& pl) {
    CountArgs& a = pl.a;
    const int n1 = b->n1;
    const double ec = em.ec, ec64 = em.ec64;
    const double s3 = std::sqrt(3.0);
    const double Re = pl.rmax * 1.01 + 1e-30;
    if (b->kind == CUTE_BIN_SIGMAPI) {
        pl.band1.resize(n1);
        for (int k = 0; k < n1; k++) {
            float lo = pl.T1[k] == 0.0 ? kBig : -(float)pl.T1[k];
            float hi = -(float)pl.T1[k + 1];
            pl.band1[k] = make_float2(lo, hi);
        }
        a.out_hi = -(float)pl.T1[n1];
        a.out_lo = pl.T1[0] == 0.0 ? kBig : -(float)pl.T1[0];
        // FP32 skip: d2_32 past top64 plus the FP32 and FP64 error of d2 at
        // that separation
        const double rt = std::sqrt(a.top64);
        a.skip32 = up32(a.top64 + 1.5 * d2_bound(rt * (1.0 + 1e-6) + 2.0 * ec, ec, ec64));
    } else {
        std::vector<float> lo_e(n1 + 1), hi_e(n1 + 1);
        for (int k = 0; k <= n1; k++) {
            const double rk = std::sqrt(pl.T1[k]);
            const double m = 1.5 * d2_bound(rk * (1.0 + 1e-6) + 2.0 * ec, ec, ec64);
            lo_e[k] = pl.T1[k] == 0.0 ? -1.0f : up32(pl.T1[k] + m);
            const double h = pl.T1[k] - m;
            hi_e[k] = h > 0.0 ? dn32(h) : -1.0f;
        }
        // bin k certifies lo_e[k] <= v < hi_e[k+1]; the kernel tests
        // med3(v, lo, hi') == v with hi' the largest float below hi_e[k+1],
        // and a band that holds no float is (inf, inf), which no v equals
        pl.band1.resize(n1);
        for (int k = 0; k < n1; k++) {
            const float lo = lo_e[k], hi = hi_e[k + 1];
            pl.band1[k] = lo < hi ? make_float2(lo, std::nextafter(hi, -INFINITY))
                                  : make_float2(INFINITY, INFINITY);
        }
        a.out_hi = lo_e[n1];
        a.out_lo = hi_e[0];
        a.skip32 = a.out_hi;
    }
    if (pl.mode == M_RMU_Z) {
        // |F - exact| <= 2 sqrt(2) ec r + 3 ec^2 + 8.1 u S, plus the FP64 terms;
        // r is bounded by the FP32 estimate r (1 + 5u) + sqrt(3) ec
        const double k1 = 2 * std::sqrt(2.0) * ec + (2 + 2 * s3) * ec64;
        // the kernel uses delta = dA0 + dA1 r with the v term folded in:
        // A2 v <= A2 Re r for every pair whose mu decision counts (r < Re)
        const double a2 = 1.5 * (8.1 * kU32 + 16 * kU64) * 1.0001;
        const double A1 = (1.5 * k1 * (1 + 8 * kU32) + a2 * Re) * 1.0001;
        const double A0 = 1.5 * (k1 * s3 * ec + 3 * ec * ec + 4 * ec64 * ec64) * 1.0001;
        a.dA1 = (float)A1;
        a.dA0 = (float)A0;
        a.dA2 = 0.0f;
        // with linear r bins the kernel evaluates dA1 ts + dA0p, ts = fl(r + s1):
        // dA0p = dA0 - dA1 s1, plus dA1 times the rounding of ts (<= u (r + |s1|),
        // of which u r is inside dA1's margin)
        if (pl.est == E_LIN)
            a.dA0p = up32(A0 - A1 * (double)a.s1 + 2.0 * kU32 * A1 * std::fabs((double)a.s1));
        else
            a.dA0p = up32(A0);
        // the decisions in bin units (E_MUF): mu always, r with linear bins
        a.rB0 = -1.0f;
        if (!a.d2_generic && !a.d2_partial && (pl.est != E_LIN || r_space_band(b, em, pl)))
            mu_space_band(b, em, pl);
    } else if (pl.mode == M_RMU_MID || pl.mode == M_SIGMAPI) {
        midpoint_bands(b, em, pl);
    }
}

// LDS of a count workgroup of kWgWaves waves: tables, the shared 64-bit
// histogram, per-wave queues and span buffers (plus extra bytes). About 40 KB
// per workgroup keeps four workgroups (16 waves) on a CU; the copies of the
// histogram are cut to fit, then the budget is relaxed for very large
// histograms (fewer workgroups per CU).
cute_status plan_lds(Plan& pl, size_t extra) {
    CountArgs& a = pl.a;
    const int n1 = a.n1, n2 = a.n2, nbins = a.nbins;
    const size_t tables = 8 * (size_t)(n1 + 1) + 8 * (size_t)(n2 + 1) + 8 * (size_t)n1 +
                          8 * (size_t)std::max(n2, 1);
    const size_t per_wave = 12 * (size_t)kQCap + 16 + 12 * (size_t)kSpanCap;
    // extra: the kernel's control words after the span buffers, plus the
    // budget word of a 32-bit histogram; a 32-bit histogram's bytes are
    // rounded up to 8
    const bool h32 = h32_mode(pl.mode);
    const size_t es = h32 ? 4 : 8;   // bytes per counter
    const size_t fixed = tables + (size_t)kWgWaves * per_wave + extra + (h32 ? 16 : 0);
    const size_t pad = h32 ? 4 : 0;
    int C = 0;
    for (size_t budget : {(size_t)40 * 1024, (size_t)80 * 1024, (size_t)160 * 1024}) {
        if (fixed + pad + es * (size_t)nbins > budget) continue;
        size_t cmax = (budget - fixed - pad) / (es * (size_t)nbins);
        C = 1;
        while (C * 2 <= (int)std::min<size_t>(cmax, 32)) C *= 2;
        break;
    }
    if (C == 0) return fail(CUTE_E_UNSUPPORTED, "histogram does not fit in LDS");
    a.copies = C;
    a.hist_words = nbins * C;
    a.hs2 = (int)es * C;
    a.hs1 = a.n2p1 * (int)es * C;
    a.h32_report = 1u << 20;
    a.h32_flush = 1u << 30;
    if (const char* t = std::getenv("CUTE_TEST_H32_FLUSH")) {
        // test hook: a small flush threshold, so that the moves of a 32-bit
        // histogram to the global counts happen many times in one count
        const long v = std::strtol(t, nullptr, 10);
        if (v > 0 && v < (1l << 30)) {
            a.h32_flush = (uint32_t)v;
            a.h32_report = std::max<uint32_t>(1u, (uint32_t)v / 4u);
        }
    }
    pl.lds = fixed + ((es * (size_t)a.hist_words + 7) & ~(size_t)7);
    return CUTE_OK;
}

void apply_item(const ItemGeom& g, CountArgs* a) {
    a->A = g.A;
    a->B = g.B;
    a->geom = g.geom;
    a->is_auto = g.is_auto;
    a->periodic = g.periodic;
    a->L = g.L;
    a->Rs = g.Rs;
    a->th_s = g.th_s;
    a->sin_th_s = g.sin_th_s;
    a->offx = g.offx;
    a->offy = g.offy;
    a->offz = g.offz;
    a->lcx = g.lcx;
    a->lcy = g.lcy;
    a->lcz = g.lcz;
}

}  // namespace cute
