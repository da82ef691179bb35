/*
 * cute.h - C ABI of the MI355X (gfx950) binned pair counter.
 *
 * The library computes the pair-count histograms DD, DR and RR that the
 * two-point correlation estimators of Alonso, "CUTE solutions for two-point
 * correlation functions from large cosmological datasets" (arXiv:1210.1833),
 * are built from:
 *
 *   N_p(bin) = number of pairs (i, j), i != j, whose separation falls in bin
 *                                                   (Sec. 2.2, eq. for N_p^d)
 *
 * for the isotropic separation r, the (r, mu) and (sigma, pi) coordinates of
 * Sec. 2.1 (pi = r mu, sigma = sqrt(r^2 - pi^2)) and the angle theta on the
 * sphere (cos theta = n1 . n2, Sec. 2.1). Candidate pairs are restricted by a
 * cell list ("chaining mesh") around each cell, or by spherical pixels for
 * the angle (Sec. 3.3). The counts feed the natural, Landy-Szalay and
 * periodic-box estimators (Sec. 2.2) and the Legendre multipoles (Sec. 2.1).
 *
 * Conventions shared by every entry point
 *  - Every function returns a cute_status and never aborts or exits. A
 *    failed call leaves its outputs unspecified and sets a thread-local
 *    message readable with cute_last_error().
 *  - Coordinates are float64 SoA arrays. Positions are comoving 3-D
 *    coordinates with the observer at the origin; for CUTE_GEOM_SPHERE they
 *    are unit vectors.
 *  - Bins are half-open [e_k, e_{k+1}); the last mu bin is closed at mu = 1.
 *  - An autocorrelation (b == NULL or b == a) counts each unordered pair i < j
 *    once and never i == j; a cross-correlation counts all n_a * n_b pairs.
 *    With these conventions the Landy-Szalay coefficient (N_r - 1)/N_d of
 *    Sec. 2.2 is exact.
 *  - Counts are exact: every pair is classified by the same FP64 squared-edge
 *    predicates as a plain FP64 double loop (mu, pi and sigma through
 *    products, theta through the chord 2 sin(theta/2)); the FP32 fast path
 *    re-tests in FP64 every pair within a proven rounding band of a decision.
 *  - Pointers are host pointers unless a flag below says otherwise. The
 *    caller owns every array it passes; the library owns grids.
 *  - All device work of a call is issued on the given stream (NULL = the
 *    null stream) and the call returns after that work has finished, except
 *    cute_batch_run, which only enqueues (and copies to device memory, which
 *    stay ordered on the stream), and cute_build_grid, which returns once the
 *    build is enqueued: every later call that takes the grid, on any stream,
 *    orders its device work after the build (a device-side wait, no host
 *    wait), and cute_get_grid_info waits for the build to report its time.
 */
#ifndef CUTE_H
#define CUTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CUTE_OK = 0,
    CUTE_E_INVALID_ARG = 1,   /* bad pointer, size, edge table or geometry    */
    CUTE_E_UNSUPPORTED = 2,   /* valid request this library does not handle   */
    CUTE_E_OUT_OF_MEMORY = 3, /* a device or host allocation failed           */
    CUTE_E_DEVICE = 4,        /* a HIP call failed (no GPU, launch failure)   */
    CUTE_E_INTERNAL = 5       /* an internal consistency check failed         */
} cute_status;

typedef enum {
    CUTE_GEOM_BOX_PERIODIC = 0, /* cube [0, L)^3, minimum-image separations
                                   (the periodic estimator of Sec. 2.2)      */
    CUTE_GEOM_BOX_OPEN = 1,     /* open catalog; cells cover its bounding box */
    CUTE_GEOM_SPHERE = 2        /* unit vectors; pixels in (cos theta, phi),
                                   the "spherical cubes" of Sec. 3.3          */
} cute_geometry;

typedef enum {
    CUTE_BIN_MONO = 0,    /* r                                   (Sec. 2.1) */
    CUTE_BIN_RMU = 1,     /* r outer, mu = |cos| in [0,1] inner  (Sec. 2.1) */
    CUTE_BIN_SIGMAPI = 2, /* sigma outer, pi inner               (Sec. 2.1) */
    CUTE_BIN_THETA = 3    /* angle theta in radians              (Sec. 2.1) */
} cute_bin_kind;

typedef enum {
    CUTE_LOS_Z = 0,        /* line of sight along +z (plane-parallel)        */
    CUTE_LOS_MIDPOINT = 1  /* along p + q, observer at the origin            */
} cute_los;

typedef enum {
    CUTE_PREC_FP64 = 0,      /* every pair classified in FP64                 */
    CUTE_PREC_FP32_EDGE = 1, /* FP32 separations; pairs inside the rounding
                                band of an edge are re-tested in FP64. Same
                                counts as CUTE_PREC_FP64.                     */
    CUTE_PREC_FP32_ONLY = 2  /* FP32 decisions only, no re-test (not exact;
                                for measuring the FP32 miscount rate)         */
} cute_precision;

typedef enum {
    CUTE_EST_NATURAL = 0, /* N_r(N_r-1)/(N_d(N_d-1)) DD/RR - 1    (Sec. 2.2) */
    CUTE_EST_LS = 1,      /* Landy-Szalay                         (Sec. 2.2) */
    CUTE_EST_BOX = 2      /* periodic box, uniform expectation    (Sec. 2.2) */
} cute_estimator;

typedef struct {
    cute_geometry geom;
    double box_size;   /* L (CUTE_GEOM_BOX_PERIODIC only); points in [0, L)  */
    double r_max;      /* largest separation (radians for SPHERE) the grid
                          will be counted at; 0 = unknown. Used to size cells
                          and, for a periodic box, to keep the stencil free
                          of duplicate images: a tile and its reach need at
                          least 3 / (1 - 2 r_max / L) + 1 cells per axis
                          (at most 406), so periodic counts reach up to
                          about r_max = 0.496 L.                              */
    double cell_size;  /* cell side (pixel side in radians for SPHERE);
                          0 = chosen by the library                           */
    int32_t device_ptrs; /* nonzero: x, y, z are device pointers             */
    int32_t tile_points; /* most points in one home tile when this grid is the
                            first argument of a count, 1..64; 0 = 64, halved
                            (down to 16) by cute_count_pairs and
                            cute_count_radial while the count has fewer tiles
                            than two per wave slot of the GPU              */
} cute_grid_params;

typedef struct {
    cute_bin_kind kind;
    cute_los los;             /* RMU: Z or MIDPOINT; SIGMAPI: MIDPOINT       */
    int32_t n1;               /* bins of r | sigma | theta                   */
    const double* edges1;     /* n1+1 strictly increasing, >= 0, finite;
                                 theta in radians, <= pi                      */
    int32_t n2;               /* bins of mu | pi; 0 for MONO and THETA       */
    const double* edges2;     /* n2+1 strictly increasing; mu within [0, 1]  */
} cute_binning;

typedef struct {
    uint64_t pair_evals;      /* candidate pairs evaluated by the kernels    */
    uint64_t pairs_in_range;  /* sum of the counts (weighted for pixel maps) */
    uint64_t retests;         /* pairs re-tested in FP64 (FP32_EDGE)         */
    uint64_t flips;           /* re-tested pairs whose FP32 decision differed
                                 from the FP64 one (the FP32-only miscounts) */
    uint64_t tiles;           /* home tiles processed                        */
    double ms_count;          /* device time of the counting launch(es)      */
} cute_count_stats;

typedef struct {
    int64_t n;                /* points                                      */
    int32_t dims[3];          /* cells per axis (SPHERE: phi, cos theta, 1)  */
    double cell[3];           /* cell sides                                  */
    double origin[3];         /* lower corner of cell (0, 0, 0)              */
    double ms_build;          /* device time of the build                    */
} cute_grid_info;

typedef struct cute_grid cute_grid;

/* Build the cell list of Sec. 3.3 over n points: cells of side a (or pixels
 * of the sphere) are assigned, the points are sorted by cell, and sorted
 * FP64 and origin-shifted FP32 copies plus cell offsets are kept on the
 * device. x, y, z: n float64 each (host, or device if p->device_ptrs).
 * The call waits once, for the bounding box and the input checks (host
 * inputs are copied by then); the rest of the build runs on `stream` after
 * it returns, so device inputs must stay valid until work that follows the
 * build on `stream` (or any call that takes the grid) has finished.
 * n may be 0. *out receives a new grid on success (free with cute_free_grid).
 * Errors: CUTE_E_INVALID_ARG for NULL pointers, n < 0 or n >= 2^31,
 * non-finite coordinates, periodic coordinates outside [0, L), vectors that
 * are not unit length (|v|^2 - 1 > 1e-6) for SPHERE, a non-positive L or a
 * negative cell size; CUTE_E_OUT_OF_MEMORY / CUTE_E_DEVICE from HIP. */
cute_status cute_build_grid(const double* x, const double* y, const double* z, int64_t n,
                            const cute_grid_params* p, void* stream, cute_grid** out);

/* Release a grid (NULL is accepted). The grid must not be in use. */
void cute_free_grid(cute_grid* g);

/* Describe a grid. */
cute_status cute_get_grid_info(const cute_grid* g, cute_grid_info* info);

/* Pixel map of an angular catalog, for the pixelised angular correlation
 * (Sec. 3.4, angular correlation function): the objects are binned into
 * equal-area pixels and every non-empty pixel becomes one point at its
 * centre whose weight is its occupancy. Counting two pixel maps with
 * cute_count_pairs adds n_p * n_q per pixel pair, which equals counting the
 * objects with each one moved to the centre of its pixel.
 * Pixels (the (cos theta, phi) pixelisation of Sec. 3.3): n_cth rings of
 * equal width in cos theta = z, n_phi sectors of equal width in phi; pixel id
 * = ring * n_phi + sector. Both integers are decided in FP64, each operation
 * rounded once:
 *   ring   = floor((z + 1) * (0.5 * n_cth)), clamped to [0, n_cth - 1];
 *   sector = the k with y*c_k - x*s_k >= 0 and y*c_{k+1} - x*s_{k+1} < 0
 *            (k + 1 taken mod n_phi), where (c_k, s_k) are the C library's
 *            cos and sin of (2 pi * k) / n_phi; sector 0 when x*x + y*y == 0.
 * The centre of pixel (r, k) is (s_r cos f_k, s_r sin f_k, c_r) with
 * c_r = (2r + 1) / n_cth - 1, s_r = sqrt((1 - c_r) * (1 + c_r)),
 * f_k = (2 pi * (k + 0.5)) / n_phi.
 * x, y, z: n unit vectors (FP64, |p|^2 within 1e-6 of 1), host or device
 *   memory as p->device_ptrs says; p->geom must be CUTE_GEOM_SPHERE, and
 *   p->r_max, cell_size and tile_points grid the centres as cute_build_grid
 *   does. cute_get_grid_info's n is the number of non-empty pixels.
 * Counting: a pixel map pairs only with another pixel map, under a THETA
 *   binning; an autocorrelation adds the n_p (n_p - 1) / 2 object pairs
 *   inside each pixel to the first bin when edges1[0] == 0 (they sit at zero
 *   separation). Batched and jackknife counts reject pixel maps.
 * Synchronous on stream, like cute_build_grid. The map is released with
 * cute_free_grid.
 * Errors: CUTE_E_INVALID_ARG for a NULL pointer, n outside [0, 2^31), a
 * geometry other than SPHERE, n_cth < 1, n_phi < 8, n_cth * n_phi >= 2^31 or
 * an input that is not a finite unit vector; those of cute_build_grid. */
cute_status cute_build_pixel_map(const double* x, const double* y, const double* z, int64_t n,
                                 int32_t n_cth, int32_t n_phi, const cute_grid_params* p,
                                 void* stream, cute_grid** out);

/* The non-empty pixels of a pixel map in ascending id order: ids[k] and
 * counts[k] (host memory, cute_get_grid_info's n entries each; either may be
 * NULL). Waits for stream. Errors: CUTE_E_INVALID_ARG for a grid that is not
 * a pixel map. */
cute_status cute_pixel_map_read(const cute_grid* g, uint32_t* ids, uint32_t* counts, void* stream);

/* Pair counts of Sec. 2.2 between grids a and b.
 * b == NULL or b == a: autocorrelation of a (pairs i < j, Sec. 2.2).
 * counts: n1 * max(n2, 1) uint64, row-major with edges1 outer, OVERWRITTEN
 * (a device pointer if counts_on_device != 0). st may be NULL.
 * Errors: CUTE_E_INVALID_ARG for bad edges, THETA on a non-SPHERE grid or a
 * 3-D kind on a SPHERE grid, grids of different geometry, a periodic r_max
 * >= L/2 or a periodic grid too coarse for r_max (rebuild it with r_max set);
 * CUTE_E_UNSUPPORTED for SIGMAPI with LOS_Z and MIDPOINT in a periodic box.
 * Pixel maps (cute_build_pixel_map) are counted with weights: see there;
 * CUTE_E_INVALID_ARG for a pixel map against a plain grid, CUTE_E_UNSUPPORTED
 * for a pixel map under a binning other than THETA; CUTE_E_INTERNAL if the
 * library's own checks on its work list fail (a tile left out).
 * Waits for stream: counts (host or device) and st are complete on return. */
cute_status cute_count_pairs(const cute_grid* a, const cute_grid* b, const cute_binning* bins,
                             cute_precision prec, uint64_t* counts, int32_t counts_on_device,
                             cute_count_stats* st, void* stream);

/* ---- Counting without allocation ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * count as cute_count_pairs (same arguments, counts, statistics and errors,
 * and it also waits for its stream), with every device temporary of the call
 * (threshold and band tables, kernel arguments, counters, the home tiles and
 * their ordering) in one fixed scratch array of CUTE_NOALLOC_SCRATCH_BYTES
 * per GPU, which the library holds from the first call on that GPU until the
 * process ends. The call allocates no device or pinned host memory: its few
 * host copies go through pageable memory. The home tiles are always built
 * without a host wait and never cut shorter for small counts.
 * Every call on one GPU uses the same array and leaves the last call's
 * contents there; each call clears the counters it needs before its kernels
 * run. Calls that overlap on one GPU (two host threads or two streams) race
 * on the array: the caller must serialise them.
 * Errors: those of cute_count_pairs; CUTE_E_INVALID_ARG, before any work is
 * enqueued, when the count's temporaries exceed the array (about 64 bytes
 * per home-tile slot of grid a plus the tables: a 2e7-point grid of 64-point
 * tiles fits). */
#define CUTE_NOALLOC_SCRATCH_BYTES (32u << 20)
cute_status cute_count_pairs_noalloc(const cute_grid* a, const cute_grid* b,
                                     const cute_binning* bins, cute_precision prec,
                                     uint64_t* counts, int32_t counts_on_device,
                                     cute_count_stats* st, void* stream);

/* Radial correlation counts (Sec. 2.1, the radial 2PCF; Sec. 3.4): the pairs
 * of objects aligned with the line of sight, i.e. subtending an angle below
 * the aperture, binned by the difference of their redshifts.
 * a, b: SPHERE grids of unit vectors (b == NULL or b == a: autocorrelation of
 *   a, pairs i < j); build them with r_max >= aperture for a tight stencil.
 * ra, rb: one redshift per object (or any per-object scalar, such as the
 *   comoving distance, to bin its difference), in the order the coordinates
 *   were given to cute_build_grid (host or device memory as r_on_device says;
 *   rb unused for an autocorrelation); finite.
 * aperture: radians in (0, pi]; a pair is aligned when its chord^2, formed
 *   from the FP64 differences of the unit vectors, is below
 *   (2 sin(aperture / 2))^2, i.e. theta < aperture.
 * edges: n_bins + 1 finite, non-negative, strictly increasing redshift
 *   differences; a pair with dz = |r_i - r_j| (one FP64 subtraction) is
 *   counted in bin k when edges[k] <= dz < edges[k + 1].
 * counts: n_bins uint64, OVERWRITTEN (a device pointer if counts_on_device).
 * FP64 throughout: few pairs fall inside an aperture, so no FP32 path.
 * Errors: CUTE_E_INVALID_ARG for NULL pointers, bad edges or aperture,
 * non-SPHERE grids or non-finite redshifts; CUTE_E_UNSUPPORTED for pixel
 * maps; those of cute_count_pairs otherwise. */
cute_status cute_count_radial(const cute_grid* a, const double* ra, const cute_grid* b,
                              const double* rb, int32_t r_on_device, double aperture,
                              int32_t n_bins, const double* edges, uint64_t* counts,
                              int32_t counts_on_device, cute_count_stats* st, void* stream);

/* Choose the cell side and the home-tile size of a grid by measurement. The
 * best cell side is data dependent (Sec. 3.3), so each candidate pair is
 * timed: a grid of n points (x, y, z, read as for cute_build_grid with
 * parameters p, cell_size and tile_points ignored) is built with it and the
 * autocorrelation under bins is counted (an evenly spread sample of about
 * 32768 home tiles when there are more, enough for several per wave, its
 * time scaled by the sampled share of the tiles), twice, keeping the faster
 * run.
 * cells: n_cell sides (0 = the library's density rule); n_cell == 0 uses
 *   {0, r/2, r/3, r/4, r/5, r/6} with r the binning's reach (theta in
 *   radians for SPHERE).
 * tiles: n_tile tile sizes in 1..64; n_tile == 0 uses {32, 64}.
 * best_cell, best_tile: the fastest pair, or, among the pairs within 2 % of
 *   the fastest time (run-to-run noise), the one with the largest tile size
 *   and then the first cell side in the candidate order. ms (nullable): the time of each
 *   pair, cell-major (n_cell x n_tile entries with the defaults' counts when
 *   0 is given; NaN for a pair the geometry rejects).
 * Errors: those of cute_build_grid and cute_count_pairs; CUTE_E_INVALID_ARG
 * for NULL outputs, n_cell or n_tile outside [0, 64], negative sides, tile
 * sizes outside 1..64, or when no pair is usable. */
cute_status cute_tune_grid(const double* x, const double* y, const double* z, int64_t n,
                           const cute_grid_params* p, const cute_binning* bins,
                           cute_precision prec, int32_t n_cell, const double* cells,
                           int32_t n_tile, const int32_t* tiles, void* stream, double* best_cell,
                           int32_t* best_tile, double* ms);

/* ---- Batched counts ---------------------------------------------------------
 * The error analyses of Sec. 4 (Fig. 5) need the same pair counts over many
 * catalogs: hundreds of mock catalogs, or one catalog with one region left out
 * at a time (jackknife). A batch counts many items in one persistent launch per
 * distinct binning; all launches of a batch are captured once in a HIP graph.
 *
 * One item: the pairs between grids a and b (b NULL or a: the autocorrelation
 * of a, pairs i < j) in which neither point is masked, binned by *bins. The
 * counts equal those of cute_count_pairs on the catalogs with the masked points
 * removed (bit-exact for FP64 and FP32_EDGE).
 * mask_a: NULL, or a->n bytes in a's input order; a nonzero byte leaves the
 *   point out. Read when the batch is created (later changes are not seen).
 * mask_b: the same for b; ignored for an autocorrelation (mask_a applies to
 *   both sides).
 * masks_on_device: nonzero if the masks are device pointers. */
typedef struct {
    const cute_grid* a;
    const cute_grid* b;
    const uint8_t* mask_a;
    const uint8_t* mask_b;
    int32_t masks_on_device;
    const cute_binning* bins;
} cute_batch_item;

typedef struct cute_batch cute_batch;

/* Plan a batch: validate every item (the errors of cute_count_pairs, plus
 * CUTE_E_INVALID_ARG for n_items < 1 or a NULL item field), build the home
 * tiles, convert the masks, order the work by estimated cost (largest item
 * first), allocate the device counts and capture the launches in a graph.
 * The grids must stay alive and unchanged until cute_batch_free. stream is
 * used for the set-up work, which is complete when the call returns. */
cute_status cute_batch_create(const cute_batch_item* items, int32_t n_items,
                              cute_precision prec, void* stream, cute_batch** out);

/* Count every item into the batch's device counts (overwritten) on stream.
 * flags: CUTE_BATCH_GRAPH launches the captured graph; CUTE_BATCH_EAGER
 * enqueues the same kernels directly (capturable by the caller: no
 * allocation, no memset, no synchronisation). Asynchronous. Runs of one batch
 * must not overlap (they share the counts). */
enum { CUTE_BATCH_GRAPH = 0, CUTE_BATCH_EAGER = 1 };
cute_status cute_batch_run(cute_batch* b, int32_t flags, void* stream);

/* Copy the counts of item (n1 * max(n2, 1) uint64), or of every item
 * concatenated in item order if item == -1, to out (device memory if
 * on_device). Synchronises stream when out is host memory. */
cute_status cute_batch_counts(const cute_batch* b, int32_t item, uint64_t* out, int32_t on_device,
                              void* stream);

/* Number of count words of item (or of all items if item == -1), and the
 * offset of item's counts in the concatenation. */
cute_status cute_batch_layout(const cute_batch* b, int32_t item, int64_t* words, int64_t* offset);

/* Work counters of the last run of item (or the sum over items if
 * item == -1): pair_evals, pairs_in_range, retests, flips, tiles; ms_count is
 * 0 (time runs with events on the stream). Synchronises stream.
 * CUTE_E_INTERNAL if a run left tiles unprocessed. */
cute_status cute_batch_stats(const cute_batch* b, int32_t item, cute_count_stats* st, void* stream);

/* Release a batch (NULL is allowed). Waits for the device. */
void cute_batch_free(cute_batch* b);

/* One-shot batch: create, run once, copy each item's counts to counts[i]
 * (device pointers if counts_on_device), free. st (nullable) receives the sum
 * over items, with ms_count the device time of the run. */
cute_status cute_count_pairs_batched(const cute_batch_item* items, int32_t n_items,
                                     cute_precision prec, uint64_t* const* counts,
                                     int32_t counts_on_device, cute_count_stats* st,
                                     void* stream);

/* ---- Jackknife by region decomposition ---------------------------------------
 * Jackknife error bars need the autocorrelation of the catalog with one
 * region left out, for each of K regions (the pair counts of Sec. 2.2 on K
 * sub-catalogs). Here all of them come from two passes over the grid,
 * whatever K: the total, and
 * one full-stencil pass that finds for each region k the pairs with at least
 * one point in it (T_k); then jack_k = total - T_k. The counts equal those of
 * cute_count_pairs on each catalog without region k (bit-exact for FP64 and
 * FP32_EDGE).
 * g: a 3-D grid (BOX_OPEN or BOX_PERIODIC). region: g's n labels in its input
 * order, each in [0, K) (device pointer if regions_on_device). K: 1..65535.
 * total: n1 * max(n2, 1) uint64 (host), the autocorrelation of g.
 * jack: K * n1 * max(n2, 1) uint64 (host), row k = catalog without region k.
 * st (nullable): both passes together.
 * Errors: CUTE_E_INVALID_ARG for NULL pointers, K out of range or a label
 * outside [0, K); CUTE_E_UNSUPPORTED for a SPHERE grid or a stencil too large
 * to tabulate; the errors of cute_count_pairs. */
cute_status cute_count_jackknife(const cute_grid* g, const int32_t* region, int32_t regions_on_device,
                                 int32_t K, const cute_binning* bins, cute_precision prec,
                                 uint64_t* total, uint64_t* jack, cute_count_stats* st,
                                 void* stream);

/* The same for a cross-correlation (DR of the Landy-Szalay estimator, Sec.
 * 2.2): jack_k counts the pairs between a without its region-k points and b
 * without its region-k points. Three passes whatever K: the total, the pairs
 * whose a point lies in region k (a's points as home), and the pairs whose b
 * point lies in region k and whose a point does not (b's points as home);
 * T_k is their sum and jack_k = total - T_k. Bit-exact like
 * cute_count_pairs on each pair of catalogs.
 * a, b: two different 3-D grids of one geometry kind; region_a, region_b:
 * their labels in input order, each in [0, K) (device pointers if
 * regions_on_device). total: the cross count of a and b; jack: K rows.
 * Errors: those of cute_count_jackknife; CUTE_E_INVALID_ARG if a == b. */
cute_status cute_count_jackknife_cross(const cute_grid* a, const int32_t* region_a,
                                       const cute_grid* b, const int32_t* region_b,
                                       int32_t regions_on_device, int32_t K,
                                       const cute_binning* bins, cute_precision prec,
                                       uint64_t* total, uint64_t* jack, cute_count_stats* st,
                                       void* stream);

/* Estimator of Sec. 2.2 per bin (xi has the shape of the counts).
 * NATURAL: dd, rr; LS: dd, dr, rr; BOX: dd only (MONO binning, periodic
 * volume box_size^3, expected count N(N-1)/2 * V_shell / L^3 with the exact
 * shell volume). nd, nr >= 2. A bin whose denominator is 0 gives NaN.
 * NATURAL and LS evaluate their numerator and denominator exactly in 128-bit
 * integers and divide once; for that they need nd, nr < 2^31 and every count
 * at most the pairs it can hold (DD <= nd(nd-1)/2, DR <= nd nr,
 * RR <= nr(nr-1)/2), else CUTE_E_INVALID_ARG. */
cute_status cute_xi_estimate(cute_estimator e, const uint64_t* dd, const uint64_t* dr,
                             const uint64_t* rr, int64_t nd, int64_t nr,
                             const cute_binning* bins, double box_size, double* xi);

/* Legendre multipoles of Sec. 2.1 from xi(r, mu) on an RMU binning:
 * xi_l(r_i) = (2l+1) int_0^1 xi(r_i, mu) P_l(mu) dmu, xi constant within each
 * mu bin. ells: n_ell even, non-negative degrees. out: n_ell * n1, row-major
 * with l outer. */
cute_status cute_xi_multipoles(const double* xi_rmu, const cute_binning* bins, int32_t n_ell,
                               const int32_t* ells, double* out);

/* Host-only diagnostic: the FP32 decision constants of the midpoint line of
 * sight (SIGMAPI, or RMU with CUTE_LOS_MIDPOINT; mu, pi = r mu and
 * sigma = sqrt(r^2 - pi^2) of Sec. 2.1 measured against l = p + q), built
 * exactly as a count builds them, for a given FP32 error model. No device
 * work. It exists so that the rounding analysis behind the exact FP32 path can
 * be checked against exact arithmetic without a GPU.
 * err[4]: bounds per component on |FP32 s - s| (s = p - q), on |FP64 s - s|,
 * on |FP32 l - l| and on |FP64 l - l|.
 * band1: 2 * n1 floats, band2: 2 * n2 floats. SIGMAPI: per bin m and H, and
 * a pair is certified in the bin along that dimension when
 * |F + m ll| <= H ll - t, with F = |s x l|^2 (sigma) or (s.l)^2 (pi),
 * ll = |l|^2 and t = K1 |l| + K0 (-m is the centre of the bin's certified
 * interval of F/ll, H its half-width less the roundings of the two fmas; a
 * bin with H < 0 is never certified). RMU: band1 holds per r bin the FP32
 * bounds lo and hi' of |s|^2 (certified when lo <= |s|^2 <= hi'), band2 the
 * plain -mu_j^2 of the mu thresholds, whose band is delta below.
 * consts: 17 floats: skip32 (pairs with FP32 |s|^2 >= skip32 are out of
 * range), llg (pairs with ll < llg are never decided in FP32), K1, K0,
 * w of sigma_max, of pi_max, of sigma_0, of pi_0, the low-side flag, then the
 * mu band coefficients A0 A1 A2 B0 B1 B2 C2 C0 of
 * delta = ll (A2 v + A1 r + A0) + |l| (B2 v + B1 r + B0) + C2 v + C0.
 * Errors: CUTE_E_INVALID_ARG (bad binning, NULL, negative or non-finite
 * error bounds), CUTE_E_UNSUPPORTED (other binnings). */
cute_status cute_fp32_decision_tables(const cute_binning* bins, const double* err,
                                      float* band1, float* band2, float* consts);

/* Host-only diagnostic: the FP32 decision constants of an RMU count with the
 * z line of sight (r and mu = |dz| / r of Sec. 2.1), built exactly as a
 * count builds them for a given FP32 error model. No device work; it exists
 * so that the rounding analysis can be checked against exact arithmetic
 * without a GPU.
 * err[2]: bounds per component on |FP32 s - s| and on |FP64 s - s|
 * (s = p - q).
 * consts: 9 floats: e1a, s1, e2a, s2 (the FP32 maps x1 = fl(r + s1) e1a and
 * x2 = fl(mu + s2) e2a, bin k along a dimension being x in [k - 1/2,
 * k + 1/2)), rB0, muB1, muB0 (a pair is certified inside its r bin k when
 * |x1 - k| <= rB0, inside its mu bin j when |x2 - j| <= muB1 / r + muB0),
 * out_hi (pairs with FP32 |s|^2 >= out_hi are out of range), and the path:
 * 2 when both r and mu are decided so (linear r bins from 0, mu bins
 * linear over [0, 1]), 3 when only mu is (logarithmic r bins), 0 or 1 when
 * the count uses the band tables instead (then rB0, muB1, muB0 are not
 * used).
 * Errors: CUTE_E_INVALID_ARG (bad binning, NULL, negative or non-finite
 * error bounds), CUTE_E_UNSUPPORTED (other binnings or lines of sight). */
cute_status cute_fp32_zlos_constants(const cute_binning* bins, const double* err, float* consts);

const char* cute_status_string(cute_status s);

/* Message of the last failed call on this thread ("" if none). */
const char* cute_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CUTE_H */
