/*
 * CPU FP64 oracle for binned pair counting (DD, DR, RR histograms).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file. It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes is the paper's definition of the pair count (Sec. 2.2, the
 * equation for N_p^d): for every pair of objects, the separation is formed and
 * the pair is added to the histogram bin that the separation falls in; an
 * autocorrelation excludes self-pairs. The loop structure is the plain double
 * loop of Sec. 3.1, parallelised as in Sec. 3.2.1 (one private histogram per
 * OpenMP thread, summed at the end).
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  - bins are half-open [e_k, e_{k+1}); the paper's strict inequalities on both
 *    sides would drop pairs lying exactly on an edge;
 *  - an autocorrelation counts each unordered pair once (i < j) and a
 *    cross-correlation counts all n1*n2 pairs, which is the convention under
 *    which the Landy-Szalay coefficient (N_r - 1)/N_d of Sec. 2.2 holds;
 *  - periodic boxes use the minimum-image separation (Sec. 2.2, the periodic
 *    estimator) with an explicit wrap rule;
 *  - every predicate compares squared quantities against squared edges, so no
 *    square root, division or libm call enters the per-pair decision; all
 *    arithmetic is IEEE binary64 with round-to-nearest and fused multiply-adds
 *    only where written (build with -ffp-contract=off);
 *  - mu = |cos| of the angle between the separation and the line of sight, in
 *    [0, 1]; its last bin is closed at 1. mu and pi are 0 when the separation
 *    (or the midpoint line of sight) is the zero vector;
 *  - the angle theta is classified through the chord c = 2 sin(theta/2), since
 *    c^2 = 2 - 2 cos(theta) is monotone in theta (Sec. 2.1, angular 2PCF).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_MONO = 0, OR_RMU = 1, OR_SIGMAPI = 2, OR_THETA = 3 };
enum { OR_LOS_Z = 0, OR_LOS_MID = 1 };

typedef struct {
    int kind;          /* OR_MONO, OR_RMU, OR_SIGMAPI, OR_THETA            */
    int los;           /* OR_LOS_Z or OR_LOS_MID (RMU); SIGMAPI needs MID   */
    int periodic;      /* minimum image in a cube of side L                */
    double L;
    int n1;            /* bins in r | sigma | theta (radians)              */
    const double* e1;  /* n1+1 edges                                       */
    int n2;            /* bins in mu | pi (0 for MONO and THETA)           */
    const double* e2;  /* n2+1 edges or NULL                               */
} or_binning;

/* Squared thresholds, computed once per call. */
typedef struct {
    or_binning b;
    double* t1;        /* r^2 | sigma^2 | chord^2 thresholds, n1+1 */
    double* t2;        /* mu^2 | pi^2 thresholds, n2+1             */
    double rmax;       /* largest separation that can be counted   */
} or_plan;

static double sq(double v) { return v * v; }

static int plan_init(or_plan* p, const or_binning* b) {
    memset(p, 0, sizeof(*p));
    p->b = *b;
    p->t1 = (double*)malloc(sizeof(double) * (size_t)(b->n1 + 1));
    if (!p->t1) return -1;
    for (int k = 0; k <= b->n1; k++) {
        if (b->kind == OR_THETA) {
            /* chord of the angle theta_k on the unit sphere */
            double c = 2.0 * sin(0.5 * b->e1[k]);
            p->t1[k] = c * c;
        } else {
            p->t1[k] = b->e1[k] * b->e1[k];
        }
    }
    if (b->n2 > 0) {
        p->t2 = (double*)malloc(sizeof(double) * (size_t)(b->n2 + 1));
        if (!p->t2) return -1;
        for (int k = 0; k <= b->n2; k++) p->t2[k] = b->e2[k] * b->e2[k];
    }
    if (b->kind == OR_SIGMAPI) {
        p->rmax = sqrt(sq(b->e1[b->n1]) + sq(b->e2[b->n2]));
    } else if (b->kind == OR_THETA) {
        p->rmax = 2.0 * sin(0.5 * b->e1[b->n1]);
    } else {
        p->rmax = b->e1[b->n1];
    }
    return 0;
}

static void plan_free(or_plan* p) {
    free(p->t1);
    free(p->t2);
}

/* Minimum image of a coordinate difference in a periodic cube of side L. */
static double wrap(double d, double L) {
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

/* Largest k in [0, n-1] with t[k] <= v, for t non-decreasing and t[0] <= v. */
static int last_le(const double* t, int n, double v) {
    int lo = 0, hi = n; /* invariant: t[lo] <= v, and hi == n or t[hi] > v */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (t[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

/* Largest j in [0, n-1] with num >= fl(t[j] * den), given that it holds at j=0.
 * The predicate is monotone in j because t is non-decreasing. */
static int last_ratio_ge(const double* t, int n, double num, double den) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (num >= t[mid] * den) lo = mid; else hi = mid;
    }
    return lo;
}

/* Classify one ordered pair. Returns the flattened bin (i1 * n2 + i2, or i1
 * when there is one dimension) or -1 when the pair is not counted. */
static int classify(const or_plan* p, double px, double py, double pz,
                    double qx, double qy, double qz) {
    const or_binning* b = &p->b;
    double dx = px - qx, dy = py - qy, dz = pz - qz;
    if (b->periodic) {
        dx = wrap(dx, b->L);
        dy = wrap(dy, b->L);
        dz = wrap(dz, b->L);
    }
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));

    if (b->kind == OR_MONO || b->kind == OR_THETA) {
        if (!(p->t1[0] <= d2 && d2 < p->t1[b->n1])) return -1;
        return last_le(p->t1, b->n1, d2);
    }

    if (b->kind == OR_RMU) {
        if (!(p->t1[0] <= d2 && d2 < p->t1[b->n1])) return -1;
        int ir = last_le(p->t1, b->n1, d2);
        double num, den;
        if (b->los == OR_LOS_Z) {
            num = dz * dz; /* mu^2 = dz^2 / r^2 */
            den = d2;
        } else {
            /* line of sight along the pair midpoint (observer at origin);
             * l = p + q is twice the midpoint, the factor cancels */
            double lx = px + qx, ly = py + qy, lz = pz + qz;
            double sl = fma(dz, lz, fma(dy, ly, dx * lx));
            double ll = fma(lz, lz, fma(ly, ly, lx * lx));
            if (ll == 0.0) { num = 0.0; den = 1.0; }
            else { num = sl * sl; den = d2 * ll; }
        }
        if (d2 == 0.0) { num = 0.0; den = 1.0; } /* mu := 0 at zero separation */
        const double* m2 = p->t2;
        int n2 = b->n2;
        if (!(num >= m2[0] * den)) return -1;                       /* mu < mu_0 */
        if (b->e2[n2] < 1.0 && num >= m2[n2] * den) return -1;      /* mu >= mu_n */
        int im = last_ratio_ge(m2, n2, num, den);
        return ir * n2 + im;
    }

    /* OR_SIGMAPI with the midpoint line of sight */
    {
        double lx = px + qx, ly = py + qy, lz = pz + qz;
        double sl = fma(dz, lz, fma(dy, ly, dx * lx));
        double ll = fma(lz, lz, fma(ly, ly, lx * lx));
        double cx = fma(dy, lz, -(dz * ly));
        double cy = fma(dz, lx, -(dx * lz));
        double cz = fma(dx, ly, -(dy * lx));
        double c2 = fma(cz, cz, fma(cy, cy, cx * cx));
        double sig_num, pi_num, den;
        if (ll == 0.0) { sig_num = d2; pi_num = 0.0; den = 1.0; }
        else { sig_num = c2; pi_num = sl * sl; den = ll; }
        const double* s2 = p->t1;
        const double* q2 = p->t2;
        int ns = b->n1, np = b->n2;
        /* sigma^2 = c2/ll compared as c2 >= S2*ll; pi^2 = sl^2/ll likewise */
        if (!(sig_num >= s2[0] * den)) return -1;
        if (sig_num >= s2[ns] * den) return -1;
        if (!(pi_num >= q2[0] * den)) return -1;
        if (pi_num >= q2[np] * den) return -1;
        int is = last_ratio_ge(s2, ns, sig_num, den);
        int ip = last_ratio_ge(q2, np, pi_num, den);
        return is * np + ip;
    }
}

int oracle_nbins(const or_binning* b) {
    return b->n1 * (b->n2 > 0 ? b->n2 : 1);
}

/* Classify one pair (exported for the edge-case tests). */
int oracle_classify(const or_binning* b, const double* p, const double* q) {
    or_plan pl;
    if (plan_init(&pl, b) != 0) return -2;
    int r = classify(&pl, p[0], p[1], p[2], q[0], q[1], q[2]);
    plan_free(&pl);
    return r;
}

/* Largest separation the binning can count (for window pruning). */
double oracle_rmax(const or_binning* b) {
    or_plan pl;
    if (plan_init(&pl, b) != 0) return -1.0;
    double r = pl.rmax;
    plan_free(&pl);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Brute force: every pair, as in the double loop of Sec. 3.1.               */
/* ------------------------------------------------------------------------ */
static void count_brute(const or_plan* p,
                        const double* xa, const double* ya, const double* za, int64_t na,
                        const double* xb, const double* yb, const double* zb, int64_t nb,
                        int is_auto, uint64_t* out, int nthreads) {
    int nbins = oracle_nbins(&p->b);
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < na; i++) {
            int64_t j0 = is_auto ? i + 1 : 0;
            for (int64_t j = j0; j < nb; j++) {
                int k = classify(p, xa[i], ya[i], za[i], xb[j], yb[j], zb[j]);
                if (k >= 0) h[k]++;
            }
        }
#pragma omp critical
        for (int k = 0; k < nbins; k++) out[k] += h[k];
        free(h);
    }
}

/* ------------------------------------------------------------------------ */
/* Exact 1-D window prune: a pair whose x-separation exceeds the largest     */
/* countable separation cannot be counted, so only pairs inside an x window  */
/* are classified. The window carries a 1e-9 relative margin, far above the  */
/* rounding of the FP64 differences, so no countable pair is skipped.        */
/* ------------------------------------------------------------------------ */
typedef struct { double x; int64_t i; } xkey;

static int cmp_xkey(const void* a, const void* b) {
    double u = ((const xkey*)a)->x, v = ((const xkey*)b)->x;
    if (u < v) return -1;
    if (u > v) return 1;
    int64_t s = ((const xkey*)a)->i, t = ((const xkey*)b)->i;
    return (s > t) - (s < t);
}

/* first index in sorted keys with x >= v */
static int64_t lower_bound_x(const xkey* k, int64_t n, double v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (k[mid].x < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static void count_window(const or_plan* p,
                         const double* xa, const double* ya, const double* za, int64_t na,
                         const double* xb, const double* yb, const double* zb, int64_t nb,
                         int is_auto, uint64_t* out, int nthreads) {
    const or_binning* b = &p->b;
    int nbins = oracle_nbins(b);
    double w = p->rmax * (1.0 + 1e-9);
    xkey* kb = (xkey*)malloc(sizeof(xkey) * (size_t)(nb > 0 ? nb : 1));
    for (int64_t j = 0; j < nb; j++) { kb[j].x = xb[j]; kb[j].i = j; }
    qsort(kb, (size_t)nb, sizeof(xkey), cmp_xkey);
    /* For an autocorrelation the sorted array is walked with position b > a,
     * which visits each unordered pair once. */
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < na; a++) {
            double px, py, pz, x0;
            int64_t lo, hi;
            if (is_auto) {
                int64_t i = kb[a].i;
                px = xb[i]; py = yb[i]; pz = zb[i]; x0 = kb[a].x;
                lo = a + 1;
            } else {
                px = xa[a]; py = ya[a]; pz = za[a]; x0 = px;
                lo = lower_bound_x(kb, nb, x0 - w);
            }
            hi = lower_bound_x(kb, nb, x0 + w);
            /* pieces of the window: [lo, hi) plus periodic images */
            int64_t seg[3][2];
            int ns = 0;
            if (hi > lo) { seg[ns][0] = lo; seg[ns][1] = hi; ns++; }
            if (b->periodic) {
                /* partners near the other face: x_b >= x0 + L - w */
                int64_t s = lower_bound_x(kb, nb, x0 + b->L - w);
                if (is_auto && s < a + 1) s = a + 1;
                if (s < hi) s = hi;
                if (s < nb) { seg[ns][0] = s; seg[ns][1] = nb; ns++; }
                if (!is_auto) {
                    /* x_b <= x0 - L + w */
                    int64_t e = lower_bound_x(kb, nb, x0 - b->L + w);
                    /* include ties at the bound */
                    while (e < nb && kb[e].x <= x0 - b->L + w) e++;
                    if (e > lo) e = lo;
                    if (e > 0) { seg[ns][0] = 0; seg[ns][1] = e; ns++; }
                }
            }
            for (int s2 = 0; s2 < ns; s2++) {
                for (int64_t c = seg[s2][0]; c < seg[s2][1]; c++) {
                    int64_t j = kb[c].i;
                    int k = classify(p, px, py, pz, xb[j], yb[j], zb[j]);
                    if (k >= 0) h[k]++;
                }
            }
        }
#pragma omp critical
        for (int k = 0; k < nbins; k++) out[k] += h[k];
        free(h);
    }
    free(kb);
}

/*
 * Count pairs.
 *  is_auto != 0: pairs i < j of catalog B (A is ignored), the autocorrelation.
 *  is_auto == 0: all pairs (i in A, j in B).
 *  prune   != 0: use the exact x-window prune instead of all pairs.
 * counts (nbins uint64) is overwritten. Returns 0, or -1 on a bad argument.
 */
int oracle_count(const double* xa, const double* ya, const double* za, int64_t na,
                 const double* xb, const double* yb, const double* zb, int64_t nb,
                 int is_auto, const or_binning* b, int prune, int nthreads,
                 uint64_t* counts) {
    if (!b || !counts || b->n1 < 1 || nb < 0 || na < 0) return -1;
    if ((b->kind == OR_RMU || b->kind == OR_SIGMAPI) && (b->n2 < 1 || !b->e2)) return -1;
    if (b->kind == OR_SIGMAPI && b->los != OR_LOS_MID) return -1;
    if (b->periodic && !(b->L > 0.0)) return -1;
    if (nthreads < 1) nthreads = 1;
    or_plan pl;
    if (plan_init(&pl, b) != 0) return -1;
    if (b->periodic && !(pl.rmax * (1.0 + 1e-9) < 0.5 * b->L)) { plan_free(&pl); return -1; }
    memset(counts, 0, sizeof(uint64_t) * (size_t)oracle_nbins(b));
    if (is_auto) { xa = xb; ya = yb; za = zb; na = nb; }
    if (prune)
        count_window(&pl, xa, ya, za, na, xb, yb, zb, nb, is_auto, counts, nthreads);
    else
        count_brute(&pl, xa, ya, za, na, xb, yb, zb, nb, is_auto, counts, nthreads);
    plan_free(&pl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pixelised angular correlation (Sec. 3.4, angular correlation function):  */
/* the catalog is binned into a pixel map and the pixels are correlated,    */
/* each weighted by the number of objects inside it.                        */
/*                                                                          */
/* Pixels are equal-area cells in (cos theta, phi): n_cth rings of equal    */
/* width in cos theta = z and n_phi sectors of equal width in phi (the      */
/* pixelisation of Sec. 3.3). Ring and sector are integers decided in FP64  */
/* by these rules, which the GPU library follows in the same precision:     */
/*  - ring r = floor((z + 1) * (n_cth / 2)), clamped to [0, n_cth - 1];     */
/*  - sector k is the one whose boundary rays enclose the point: the point  */
/*    is on or counter-clockwise of the ray at phi_k = 2 pi k / n_phi and   */
/*    strictly clockwise of the ray at phi_{k+1}. "Counter-clockwise of the */
/*    ray with direction (c, s)" is the sign of y*c - x*s, each product and */
/*    the difference rounded once, with c = cos(phi_k), s = sin(phi_k) from */
/*    the C library. A point with x^2 + y^2 == 0 (a pole) is in sector 0.   */
/* The centre of pixel (r, k) is (s_r cos f_k, s_r sin f_k, c_r) with       */
/* c_r = (2r + 1)/n_cth - 1, s_r = sqrt((1 - c_r)(1 + c_r)) and             */
/* f_k = 2 pi (k + 1/2) / n_phi. The pixel id is r * n_phi + k.             */
/* ------------------------------------------------------------------------ */
static const double OR_TWO_PI = 6.283185307179586476925286766559;

static double ray_side(double x, double y, double c, double s) {
    double a = y * c;
    double b = x * s;
    return a - b;
}

/* Pixel id of every point; -1 on a bad argument or if a sector search fails. */
int oracle_pixel_ids(const double* x, const double* y, const double* z, int64_t n,
                     int n_cth, int n_phi, int64_t* ids) {
    if (n < 0 || n_cth < 1 || n_phi < 8 || (n > 0 && (!x || !y || !z || !ids))) return -1;
    double* bc = (double*)malloc(sizeof(double) * (size_t)n_phi);
    double* bs = (double*)malloc(sizeof(double) * (size_t)n_phi);
    if (!bc || !bs) { free(bc); free(bs); return -1; }
    for (int k = 0; k < n_phi; k++) {
        double a = OR_TWO_PI * (double)k / (double)n_phi;
        bc[k] = cos(a);
        bs[k] = sin(a);
    }
    int bad = 0;
    for (int64_t i = 0; i < n; i++) {
        double t = (z[i] + 1.0) * (0.5 * (double)n_cth);
        int64_t r = (int64_t)floor(t);
        if (r < 0) r = 0;
        if (r > n_cth - 1) r = n_cth - 1;
        int64_t k = 0;
        if (x[i] * x[i] + y[i] * y[i] != 0.0) {
            /* start from the sector of atan2, then step to the enclosing one */
            double f = atan2(y[i], x[i]);
            if (f < 0.0) f += OR_TWO_PI;
            k = (int64_t)floor(f / OR_TWO_PI * (double)n_phi);
            k = ((k % n_phi) + n_phi) % n_phi;
            int found = 0;
            for (int it = 0; it < 4 && !found; it++) {
                int64_t k1 = (k + 1) % n_phi;
                if (ray_side(x[i], y[i], bc[k], bs[k]) < 0.0) k = (k + n_phi - 1) % n_phi;
                else if (ray_side(x[i], y[i], bc[k1], bs[k1]) >= 0.0) k = k1;
                else found = 1;
            }
            if (!found) bad = 1;
        }
        ids[i] = r * (int64_t)n_phi + k;
    }
    free(bc);
    free(bs);
    return bad ? -1 : 0;
}

/* Centres of the pixels with the given ids (unit vectors, FP64). */
int oracle_pixel_centres(const int64_t* ids, int64_t n, int n_cth, int n_phi,
                         double* x, double* y, double* z) {
    if (n < 0 || n_cth < 1 || n_phi < 8) return -1;
    for (int64_t i = 0; i < n; i++) {
        if (ids[i] < 0 || ids[i] >= (int64_t)n_cth * n_phi) return -1;
        int64_t r = ids[i] / n_phi, k = ids[i] % n_phi;
        double c = (double)(2 * r + 1) / (double)n_cth - 1.0;
        double s = sqrt((1.0 - c) * (1.0 + c));
        double f = OR_TWO_PI * ((double)k + 0.5) / (double)n_phi;
        x[i] = s * cos(f);
        y[i] = s * sin(f);
        z[i] = c;
    }
    return 0;
}

/*
 * Weighted pair counts: every pair (i, j) adds w_i * w_j to its bin.
 *  is_auto != 0: pairs i < j of catalog B, plus the w_i (w_i - 1) / 2 pairs of
 *  objects that share a pixel, which sit at zero separation.
 *  is_auto == 0: all pairs (i in A, j in B).
 * Plain double loop (Sec. 3.1). Returns 0, or -1 on a bad argument.
 */
int oracle_count_weighted(const double* xa, const double* ya, const double* za,
                          const uint32_t* wa, int64_t na,
                          const double* xb, const double* yb, const double* zb,
                          const uint32_t* wb, int64_t nb,
                          int is_auto, const or_binning* b, int nthreads, uint64_t* counts) {
    if (!b || !counts || b->n1 < 1 || nb < 0 || na < 0) return -1;
    if ((b->kind == OR_RMU || b->kind == OR_SIGMAPI) && (b->n2 < 1 || !b->e2)) return -1;
    if (b->periodic && !(b->L > 0.0)) return -1;
    if (nthreads < 1) nthreads = 1;
    or_plan pl;
    if (plan_init(&pl, b) != 0) return -1;
    int nbins = oracle_nbins(b);
    memset(counts, 0, sizeof(uint64_t) * (size_t)nbins);
    if (is_auto) { xa = xb; ya = yb; za = zb; wa = wb; na = nb; }
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < na; i++) {
            int64_t j0 = is_auto ? i + 1 : 0;
            for (int64_t j = j0; j < nb; j++) {
                int k = classify(&pl, xa[i], ya[i], za[i], xb[j], yb[j], zb[j]);
                if (k >= 0) h[k] += (uint64_t)wa[i] * (uint64_t)wb[j];
            }
            if (is_auto) {
                int k = classify(&pl, xa[i], ya[i], za[i], xa[i], ya[i], za[i]);
                if (k >= 0) h[k] += (uint64_t)wa[i] * ((uint64_t)wa[i] - 1u) / 2u;
            }
        }
#pragma omp critical
        for (int k = 0; k < nbins; k++) counts[k] += h[k];
        free(h);
    }
    plan_free(&pl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Radial correlation (Sec. 2.1, the radial 2PCF; Sec. 3.4): pairs of       */
/* objects aligned with the line of sight, i.e. subtending an angle theta   */
/* below the aperture, binned by the difference of their redshifts.         */
/* The angle is tested through the chord as in the angular case:            */
/* theta < aperture  <=>  c^2 < (2 sin(aperture / 2))^2, with c^2 formed    */
/* from the FP64 differences of the unit vectors. The redshift difference   */
/* dz = |z_i - z_j| (one rounding) falls in bin k when e_k <= dz < e_{k+1}. */
/* ------------------------------------------------------------------------ */
int oracle_count_radial(const double* xa, const double* ya, const double* za, const double* ra,
                        int64_t na, const double* xb, const double* yb, const double* zb,
                        const double* rb, int64_t nb, int is_auto, double aperture, int nbins,
                        const double* edges, int nthreads, uint64_t* counts) {
    if (!counts || !edges || nbins < 1 || na < 0 || nb < 0 || !(aperture > 0.0)) return -1;
    for (int k = 0; k < nbins; k++)
        if (!(edges[k] < edges[k + 1]) || edges[k] < 0.0) return -1;
    if (nthreads < 1) nthreads = 1;
    const double c = 2.0 * sin(0.5 * aperture);
    const double t_ap = c * c;
    memset(counts, 0, sizeof(uint64_t) * (size_t)nbins);
    if (is_auto) { xa = xb; ya = yb; za = zb; ra = rb; na = nb; }
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < na; i++) {
            int64_t j0 = is_auto ? i + 1 : 0;
            for (int64_t j = j0; j < nb; j++) {
                double dx = xa[i] - xb[j], dy = ya[i] - yb[j], dz = za[i] - zb[j];
                double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (!(d2 < t_ap)) continue;
                double dr = fabs(ra[i] - rb[j]);
                if (!(edges[0] <= dr && dr < edges[nbins])) continue;
                h[last_le(edges, nbins, dr)]++;
            }
        }
#pragma omp critical
        for (int k = 0; k < nbins; k++) counts[k] += h[k];
        free(h);
    }
    return 0;
}
