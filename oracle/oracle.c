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
static inline __attribute__((always_inline)) double wrap(double d, double L) {
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

/* Largest k in [0, n-1] with t[k] <= v, for t non-decreasing and t[0] <= v.
 * A binary search with a fixed number of halvings: the answer stays in
 * [lo, lo + len) and t[lo] <= v holds throughout. */
static inline __attribute__((always_inline)) int last_le(const double* t, int n, double v) {
    int lo = 0, len = n;
    while (len > 1) {
        int half = len / 2;
        lo = (t[lo + half] <= v) ? lo + half : lo;
        len -= half;
    }
    return lo;
}

/* Largest j in [0, n-1] with num >= fl(t[j] * den), given that it holds at j=0.
 * The predicate is monotone in j because t is non-decreasing and den >= 0
 * (rounding is monotone), so the same halving search applies. */
static inline __attribute__((always_inline)) int last_ratio_ge(const double* t, int n, double num,
                                                                double den) {
    int lo = 0, len = n;
    while (len > 1) {
        int half = len / 2;
        lo = (num >= t[lo + half] * den) ? lo + half : lo;
        len -= half;
    }
    return lo;
}

/* Classify one ordered pair. Returns the flattened bin (i1 * n2 + i2, or i1
 * when there is one dimension) or -1 when the pair is not counted. Inlined
 * into each loop, which is compiled with and without the FMA instructions. */
static inline __attribute__((always_inline)) int classify(const or_plan* p, double px, double py, double pz,
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
/* The inner loop over j is a function of its own, compiled twice (with and  */
/* without the FMA instruction set, chosen at load time): fma() is correctly */
/* rounded either way, so both give the same counts; the instruction is only */
/* faster than the library call.                                             */
/* ------------------------------------------------------------------------ */
__attribute__((target_clones("fma", "default"), noinline))
static void brute_row(const or_plan* p, double px, double py, double pz,
                      const double* xb, const double* yb, const double* zb,
                      int64_t j0, int64_t nb, uint64_t* h) {
    for (int64_t j = j0; j < nb; j++) {
        int k = classify(p, px, py, pz, xb[j], yb[j], zb[j]);
        if (k >= 0) h[k]++;
    }
}

static void count_brute(const or_plan* p,
                        const double* xa, const double* ya, const double* za, int64_t na,
                        const double* xb, const double* yb, const double* zb, int64_t nb,
                        int is_auto, uint64_t* out, int nthreads) {
    int nbins = oracle_nbins(&p->b);
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < na; i++)
            brute_row(p, xa[i], ya[i], za[i], xb, yb, zb, is_auto ? i + 1 : 0, nb, h);
#pragma omp critical
        for (int k = 0; k < nbins; k++) out[k] += h[k];
        free(h);
    }
}

/* ------------------------------------------------------------------------ */
/* Exact band-and-window prune. Every countable pair has a separation below  */
/* rmax, so |dx| < rmax and |dy| < rmax (minimum image in a periodic box).   */
/* The points are grouped into bands of y, each at least w = rmax (1 + 1e-9) */
/* wide, and sorted by x inside each band; only the pairs in the same or in  */
/* adjacent bands whose x-separation is below w are classified. Two bands    */
/* two or more apart are separated by a whole band, i.e. |dy| >= w. The 1e-9 */
/* margin (and a 1e-6 one on the band width) lies far above the rounding of  */
/* the FP64 differences and of the band index, so no countable pair is       */
/* skipped; the tests check the result against the brute-force loop.         */
/* A periodic box uses cyclic bands when there are at least three, else one  */
/* band (the x window alone, with its periodic images).                       */
/* ------------------------------------------------------------------------ */
typedef struct { int band; double x; int64_t i; } bkey;

static int cmp_bkey(const void* a, const void* b) {
    const bkey* u = (const bkey*)a;
    const bkey* v = (const bkey*)b;
    if (u->band != v->band) return u->band < v->band ? -1 : 1;
    if (u->x < v->x) return -1;
    if (u->x > v->x) return 1;
    return (u->i > v->i) - (u->i < v->i);
}

typedef struct {
    int nb;             /* bands                                         */
    int cyclic;         /* bands wrap (periodic box, nb >= 3)            */
    double y0, bw;      /* band k holds y0 + k bw <= y < y0 + (k+1) bw     */
} band_geo;

static int band_of(const band_geo* g, double y) {
    double q = floor((y - g->y0) / g->bw);
    if (!(q >= 0.0)) return 0;
    if (q >= (double)(g->nb - 1)) return g->nb - 1;
    return (int)q;
}

/* Catalog B sorted by (band, x): coordinates, input index and the first    */
/* position of each band.                                                    */
typedef struct {
    double *x, *y, *z;
    int64_t* idx;
    int64_t* start;     /* nb + 1 */
} banded;

static int banded_init(banded* s, const band_geo* g, const double* x, const double* y,
                       const double* z, int64_t n) {
    memset(s, 0, sizeof(*s));
    size_t m = (size_t)(n > 0 ? n : 1);
    bkey* k = (bkey*)malloc(sizeof(bkey) * m);
    s->x = (double*)malloc(sizeof(double) * m);
    s->y = (double*)malloc(sizeof(double) * m);
    s->z = (double*)malloc(sizeof(double) * m);
    s->idx = (int64_t*)malloc(sizeof(int64_t) * m);
    s->start = (int64_t*)calloc((size_t)g->nb + 1, sizeof(int64_t));
    if (!k || !s->x || !s->y || !s->z || !s->idx || !s->start) { free(k); return -1; }
    for (int64_t j = 0; j < n; j++) { k[j].band = band_of(g, y[j]); k[j].x = x[j]; k[j].i = j; }
    qsort(k, (size_t)n, sizeof(bkey), cmp_bkey);
    for (int64_t j = 0; j < n; j++) {
        int64_t i = k[j].i;
        s->x[j] = x[i]; s->y[j] = y[i]; s->z[j] = z[i]; s->idx[j] = i;
        s->start[k[j].band + 1]++;
    }
    for (int b = 0; b < g->nb; b++) s->start[b + 1] += s->start[b];
    free(k);
    return 0;
}

static void banded_free(banded* s) {
    free(s->x); free(s->y); free(s->z); free(s->idx); free(s->start);
}

/* first position in [lo, hi) of the x-sorted run with x >= v */
static int64_t lower_x(const double* x, int64_t lo, int64_t hi, double v) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (x[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* first position in [lo, hi) with x > v */
static int64_t upper_x(const double* x, int64_t lo, int64_t hi, double v) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (x[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Jackknife regions (optional): the pair counts of the catalog without     */
/* region k are the total minus the pairs with at least one point in k, so  */
/* each counted pair also adds 1 to the histogram of every region it        */
/* touches (once when both points share the region).                        */
typedef struct {
    const int32_t* reg;  /* region of each sorted point, or NULL */
    uint64_t* touch;     /* K * nbins, this thread's               */
    int nbins;
} region_acc;

/* Classify point p against the positions [s, e) of the sorted catalog. */
/* A pair whose FP64 squared separation (formed as the classification forms  */
/* it) is at least w^2 is skipped before the classification: a counted pair */
/* has d2 < rmax^2 (1 + 13 u) < w^2 in every binning (for sigma-pi because   */
/* sigma^2 + pi^2 = r^2 for any line of sight, up to a few roundings).       */
__attribute__((target_clones("fma", "default"), noinline))
static void window_row(const or_plan* p, double px, double py, double pz, int32_t rp,
                       const banded* B, int64_t s, int64_t e, uint64_t* h, const region_acc* ra) {
    const or_binning* bn = &p->b;
    const double w = p->rmax * (1.0 + 1e-9), w2 = w * w;
    for (int64_t c = s; c < e; c++) {
        double dx = px - B->x[c], dy = py - B->y[c], dz = pz - B->z[c];
        if (bn->periodic) {
            dx = wrap(dx, bn->L);
            dy = wrap(dy, bn->L);
            dz = wrap(dz, bn->L);
        }
        if (fma(dz, dz, fma(dy, dy, dx * dx)) >= w2) continue;
        int k = classify(p, px, py, pz, B->x[c], B->y[c], B->z[c]);
        if (k < 0) continue;
        h[k]++;
        if (ra->reg) {
            int32_t rq = ra->reg[c];
            ra->touch[(size_t)rp * (size_t)ra->nbins + (size_t)k]++;
            if (rq != rp) ra->touch[(size_t)rq * (size_t)ra->nbins + (size_t)k]++;
        }
    }
}

/* All partners of p in band b of B within the x window (plus the periodic   */
/* images of the window); with from >= 0 only positions after from (the     */
/* autocorrelation inside p's own band, where from is p's position).         */
static void visit_band(const or_plan* p, double w, double px, double py, double pz, int32_t rp,
                       const banded* B, int b, int64_t from, uint64_t* h, const region_acc* ra) {
    const or_binning* bn = &p->b;
    const double* xs = B->x;
    int64_t s = B->start[b], e = B->start[b + 1];
    if (from >= 0) s = from + 1;
    if (s >= e) return;
    int64_t lo = from >= 0 ? s : lower_x(xs, s, e, px - w);
    int64_t hi = lower_x(xs, s, e, px + w);
    if (hi > lo) window_row(p, px, py, pz, rp, B, lo, hi, h, ra);
    if (!bn->periodic) return;
    /* partners near the far face: x_b >= x0 + L - w */
    int64_t s2 = lower_x(xs, s, e, px + bn->L - w);
    if (s2 < hi) s2 = hi;
    if (s2 < e) window_row(p, px, py, pz, rp, B, s2, e, h, ra);
    if (from < 0) {
        /* partners near the near face: x_b <= x0 - L + w */
        int64_t e2 = upper_x(xs, s, e, px - bn->L + w);
        if (e2 > lo) e2 = lo;
        if (e2 > s) window_row(p, px, py, pz, rp, B, s, e2, h, ra);
    }
}

static int band_geometry(const or_plan* p, const double* ya, int64_t na, const double* yb,
                         int64_t nb, band_geo* g) {
    const or_binning* b = &p->b;
    double w = p->rmax * (1.0 + 1e-9);
    g->bw = w * (1.0 + 1e-6);
    g->cyclic = 0;
    if (b->periodic) {
        g->y0 = 0.0;
        double q = floor(b->L / g->bw);
        g->nb = q >= 3.0 ? (int)(q < 1048576.0 ? q : 1048576.0) : 1;
        if (g->nb >= 3) {
            g->bw = b->L / (double)g->nb;   /* >= the width asked for */
            g->cyclic = 1;
        }
        return 0;
    }
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < na; i++) { if (ya[i] < lo) lo = ya[i]; if (ya[i] > hi) hi = ya[i]; }
    for (int64_t i = 0; i < nb; i++) { if (yb[i] < lo) lo = yb[i]; if (yb[i] > hi) hi = yb[i]; }
    if (!(hi >= lo)) { lo = hi = 0.0; }
    g->y0 = lo;
    double q = floor((hi - lo) / g->bw) + 1.0;
    if (q > 1048576.0) { g->bw = (hi - lo) / 1048575.0; q = 1048576.0; }
    g->nb = (int)q;
    return 0;
}

static int count_window(const or_plan* p,
                        const double* xa, const double* ya, const double* za, int64_t na,
                        const double* xb, const double* yb, const double* zb, int64_t nb,
                        int is_auto, uint64_t* out, int nthreads,
                        const int32_t* region, int nreg, uint64_t* touch_out) {
    int nbins = oracle_nbins(&p->b);
    double w = p->rmax * (1.0 + 1e-9);
    band_geo g;
    band_geometry(p, ya, na, yb, nb, &g);
    banded B;
    if (banded_init(&B, &g, xb, yb, zb, nb) != 0) { banded_free(&B); return -1; }
    int32_t* sreg = NULL;
    if (region) {
        sreg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb > 0 ? nb : 1));
        if (!sreg) { banded_free(&B); return -1; }
        for (int64_t j = 0; j < nb; j++) sreg[j] = region[B.idx[j]];
    }
    int fail = 0;
#pragma omp parallel num_threads(nthreads)
    {
        uint64_t* h = (uint64_t*)calloc((size_t)nbins, sizeof(uint64_t));
        region_acc ra = {sreg, NULL, nbins};
        if (sreg) ra.touch = (uint64_t*)calloc((size_t)nreg * (size_t)nbins, sizeof(uint64_t));
        if (!h || (sreg && !ra.touch)) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < (is_auto ? nb : na); a++) {
            if (fail) continue;
            double px, py, pz;
            int32_t rp = 0;
            int ba;
            if (is_auto) {
                px = B.x[a]; py = B.y[a]; pz = B.z[a];
                rp = sreg ? sreg[a] : 0;
                ba = band_of(&g, py);
                /* the own band from the next position on, then the next band */
                visit_band(p, w, px, py, pz, rp, &B, ba, a, h, &ra);
                int bn1 = ba + 1;
                if (bn1 == g.nb && g.cyclic) bn1 = 0;
                if (bn1 < g.nb && bn1 != ba) visit_band(p, w, px, py, pz, rp, &B, bn1, -1, h, &ra);
            } else {
                px = xa[a]; py = ya[a]; pz = za[a];
                ba = band_of(&g, py);
                int bands[3] = {ba - 1, ba, ba + 1}, nvis = 0;
                for (int t = 0; t < 3; t++) {
                    int bb = bands[t];
                    if (g.cyclic) bb = (bb + g.nb) % g.nb;
                    if (bb < 0 || bb >= g.nb) continue;
                    int dup = 0;
                    for (int u = 0; u < t; u++) if (bands[u] == bb) dup = 1;
                    bands[t] = bb;
                    if (dup) continue;
                    visit_band(p, w, px, py, pz, 0, &B, bb, -1, h, &ra);
                    nvis++;
                }
                (void)nvis;
            }
        }
#pragma omp critical
        {
            if (h) for (int k = 0; k < nbins; k++) out[k] += h[k];
            if (ra.touch)
                for (size_t k = 0; k < (size_t)nreg * (size_t)nbins; k++) touch_out[k] += ra.touch[k];
        }
        free(h);
        free(ra.touch);
    }
    free(sreg);
    banded_free(&B);
    return fail ? -1 : 0;
}

/*
 * Count pairs.
 *  is_auto != 0: pairs i < j of catalog B (A is ignored), the autocorrelation.
 *  is_auto == 0: all pairs (i in A, j in B).
 *  prune   != 0: use the exact band-and-window prune instead of all pairs.
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
    int rc = 0;
    if (prune)
        rc = count_window(&pl, xa, ya, za, na, xb, yb, zb, nb, is_auto, counts, nthreads,
                          NULL, 0, NULL);
    else
        count_brute(&pl, xa, ya, za, na, xb, yb, zb, nb, is_auto, counts, nthreads);
    plan_free(&pl);
    return rc;
}

/*
 * Jackknife autocorrelations by regions: for every k in [0, K), the pair
 * counts of the catalog with the points of region k left out (the counts of
 * Sec. 2.2 on K sub-catalogs). Each one equals the count of the whole
 * catalog minus the pairs with at least one point in region k, so one pass
 * over the pairs (with the exact prune) gives all of them.
 * region: n labels in [0, K). total: nbins (the whole catalog); jack: K * nbins,
 * row k = the catalog without region k. Returns 0, or -1 on a bad argument.
 */
int oracle_count_jackknife(const double* x, const double* y, const double* z, int64_t n,
                           const int32_t* region, int K, const or_binning* b, int nthreads,
                           uint64_t* total, uint64_t* jack) {
    if (!b || !total || !jack || !region || K < 1 || n < 0 || b->n1 < 1) return -1;
    if ((b->kind == OR_RMU || b->kind == OR_SIGMAPI) && (b->n2 < 1 || !b->e2)) return -1;
    if (b->kind == OR_SIGMAPI && b->los != OR_LOS_MID) return -1;
    if (b->periodic && !(b->L > 0.0)) return -1;
    for (int64_t i = 0; i < n; i++)
        if (region[i] < 0 || region[i] >= K) return -1;
    if (nthreads < 1) nthreads = 1;
    or_plan pl;
    if (plan_init(&pl, b) != 0) return -1;
    if (b->periodic && !(pl.rmax * (1.0 + 1e-9) < 0.5 * b->L)) { plan_free(&pl); return -1; }
    int nbins = oracle_nbins(b);
    memset(total, 0, sizeof(uint64_t) * (size_t)nbins);
    uint64_t* touch = (uint64_t*)calloc((size_t)K * (size_t)nbins, sizeof(uint64_t));
    if (!touch) { plan_free(&pl); return -1; }
    int rc = count_window(&pl, x, y, z, n, x, y, z, n, 1, total, nthreads, region, K, touch);
    for (size_t k = 0; k < (size_t)K; k++)
        for (size_t q = 0; q < (size_t)nbins; q++)
            jack[k * (size_t)nbins + q] = total[q] - touch[k * (size_t)nbins + q];
    free(touch);
    plan_free(&pl);
    return rc;
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
