// Internal structures shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "cute.h"

namespace cute {

// FP64 copy of a sorted point (the raw caller coordinates).
struct alignas(32) P64 {
    double x, y, z;
    uint32_t idx;   // position of the point in the caller's input order
    uint32_t pad;
};

// Sizes shared by the kernels and their launch planning.
constexpr int kQCap = 128;        // FP64 re-test queue entries per wave
constexpr int kSpanCap = 192;     // neighbour spans buffered per wave
constexpr int kWgWaves = 4;       // waves per count workgroup

// Kinds of pair classification the kernels are specialised for.
enum Mode : int { M_MONO = 0, M_RMU_Z = 1, M_RMU_MID = 2, M_SIGMAPI = 3, M_THETA = 4, M_RADIAL = 5 };
// How a bin index is estimated from the squared separation.
// Estimate flags of a count kernel: bit 0, dimension 1 (r or theta) is
// estimated from log(d2) (log-spaced edges) rather than linearly; bit 1, the
// mu decision of the z line of sight is taken in mu space (linear mu edges
// covering [0, 1]), FP32_EDGE only.
enum Est : int { E_LIN = 0, E_LOG = 1, E_MUF = 2 };
constexpr bool est_log(int e) { return (e & E_LOG) != 0; }
constexpr bool est_muf(int e) { return (e & E_MUF) != 0; }
// Precision path.
enum Prec : int { P_FP64 = 0, P_FP32E = 1, P_FP32O = 2 };

// LDS histogram counters: 32-bit for the midpoint kinds (their two-dimensional
// histograms are large, and half the bytes keeps more workgroups on a CU),
// 64-bit for the others. A 32-bit histogram is moved to the global counts
// before any counter can wrap (see h32_flush).
template <int MODE>
constexpr bool kH32 = MODE == M_SIGMAPI || MODE == M_RMU_MID;

// Workgroups per CU a count kernel is compiled for (its register budget):
// five for the one-variable FP32_EDGE kernels, four for the others.
template <int MODE, int PREC>
constexpr int kWgPerCu = (PREC == P_FP32E && (MODE == M_THETA || MODE == M_MONO)) ? 5 : 4;
constexpr bool h32_mode(int mode) { return mode == M_SIGMAPI || mode == M_RMU_MID; }

// A home tile: a run of sorted points inside one row of cells.
struct Tile {
    uint32_t start, end;  // sorted point range [start, end)
    uint32_t row;         // row index (cy + ny * cz; SPHERE: band)
    uint32_t c0c1;        // first cell (low 16 bits) and last cell (high 16 bits) along x
};

// Device-side description of a grid.
struct GridView {
    const float4* p32;        // sorted, origin-shifted FP32 (x - c, y - c, z - c, 0)
    const P64* p64;           // sorted FP64 raw coordinates
    const uint32_t* cstart;   // cell offsets, ncells + 1
    int nx, ny, nz;           // cells per axis (SPHERE: phi cells, bands, 1)
    double ox, oy, oz;        // lower corner of cell (0,0,0) (SPHERE: phi0 = 0, zmin)
    double ax, ay, az;        // cell sides (SPHERE: dphi, dz)
    double cx, cy, cz;        // FP32 origin
};

struct cute_grid_impl;

// Everything a count kernel needs, passed by value.
struct CountArgs {
    const CountArgs* self;          // a copy of these arguments in device memory
    GridView A, B;
    const Tile* tiles;
    uint32_t ntiles;
    const uint32_t* ntiles_dev;     // when set, the tile count in device memory (ntiles is
                                    // then only the capacity of tiles)
    uint32_t* work_head;            // next tile to pop (global counter)
    unsigned long long* counts;     // nbins global uint64 counts
    unsigned long long* stats;      // [0] pair evals, [1] retests, [2] flips, [3] tiles
    int geom;                       // cute_geometry
    int is_auto;
    int periodic;
    double L;
    double Rs;                      // stencil radius (with margin); SPHERE: chord
    double th_s;                    // SPHERE: angular stencil radius (radians)
    double sin_th_s;                // SPHERE: sin(th_s)
    int n1, n2, nbins;
    float n1m1, n2m1;               // n1 - 1 and n2 - 1 as floats (estimate clamps)
    int copies;                     // LDS histogram copies per wave (power of two)
    int hist_words;                 // nbins * copies (counters of 4 or 8 bytes, kH32)
    // 32-bit histograms: a wave reports its pair evaluations to the
    // workgroup's budget once it has h32_report of them, and the histogram is
    // moved to counts once the budget reaches h32_flush (< 2^31)
    uint32_t h32_report, h32_flush;
    // FP32 geometry constants
    float offx, offy, offz;         // FP32(cA - cB), added to home points (open boxes)
    float lcx, lcy, lcz;            // FP32(2 cB): l = home_eff + q + lc (midpoint LOS)
    // dimension-1 estimate: k = clamp(int(fma(t, e1a, e1b)), 0, n1-1)
    float e1a, e1b;
    // dimension-2 estimate (mu or pi), linear in mu (or pi)
    float e2a, e2b;
    int d2_generic;                 // dimension-2 edges are not linear
    int d2_partial;                 // mu range is not [0, 1] with a closed top, or pi starts > 0
    // FP32 decision constants
    float out_lo, out_hi;           // dim 1 is clean-out if v < out_lo or v >= out_hi
    float bot32, top32;             // FP32-rounded T1[0], T1[n1] (tentative decisions)
    float d2lo32, d2hi32;           // FP32-rounded T2[0], T2[n2]
    float nlo2_first, nhi2_last;    // -T2f[0] (or +BIG), -T2f[n2] (or -BIG) for dim-2 range
    // rounding band of the mu predicates, per pair. Midpoint line of sight:
    //   delta = ll (A2 v + A1 r + A0) + |l| (B2 v + B1 r + B0) + C2 v + C0;
    // z line of sight: delta = A1 r + A0 (dA0p below)
    float dA0, dA1, dA2, dB0, dB1, dB2, dC2, dC0;
    // midpoint line of sight: a pair is decided in FP32 only when
    // ll = |l|^2 >= llg (the direction of l is then known to a bounded angle)
    float llg;
    // sigma-pi: the per-edge parts of the rounding bands sit in the band
    // tables; the per-pair part is t = spK1 |l| + spK0, and a decision
    // F + w ll against +-t (F = |s x l|^2 or (s.l)^2). Out of range: sigma or
    // pi at or past its top edge (wstop, wptop), below its first edge (wsbot,
    // wpbot, tested only when sp_low)
    float spK1, spK0;
    float sp_wstop, sp_wptop, sp_wsbot, sp_wpbot;
    int sp_low;
    // tables (global; staged into LDS)
    const float2* band1;            // n1 entries: (lo_k, below(hi_{k+1})) FP32 band thresholds of dim 1
                                    // (SIGMAPI: the w of the lower and upper edges)
    const float2* band2;            // n2 entries: (-T2f[k] or +BIG, -T2f[k+1] or -BIG)
    const double* T1;               // n1+1 canonical FP64 thresholds of dim 1
    const double* T2;               // n2+1 canonical FP64 thresholds of dim 2
    int mu_top_closed;              // last mu edge == 1
    // FP32 bin estimates (biased integers, see the kernels): shifts of the
    // estimated variables, clamp tops (bits of 2^23 + n - 1), n2 or 1
    float s1, s2;
    uint32_t top1, top2;
    int n2p1;
    // LDS histogram strides in bytes: dimension 1 (n2p1 << log2 copies times
    // the counter size) and dimension 2 (copies times the counter size)
    int hs1, hs2;
    // constant term of the mu band of the z line of sight as the kernel uses
    // it (dA0 for log r bins, dA0 - dA1 s1 plus its rounding for linear ones)
    float dA0p;
    // mu in mu space (E_MUF): a pair is inside its mu bin when the offset d
    // of its position in bin units from the nearest bin centre satisfies
    // |d| <= muB1 / r + muB0 (muB1 < 0: the band grows as the separation
    // shrinks)
    float muB1, muB0;
    // r in bin units (E_MUF with linear r bins, which start at r = 0 then):
    // inside its r bin when |d| <= rB0
    float rB0;
    // precomputed neighbour rows (see ItemGeom::stencil), or nullptr
    const int4* stencil;
    int nst;
    // region pass of the jackknife (full stencil): sorted-order region of
    // each neighbour point, the home region of this item's tiles, the weights
    // of a pair whose neighbour lies in the home region (wsame) or not
    // (wdiff), and the j != i test in the home tile's own span when home and
    // neighbours are one catalog; regs == nullptr otherwise (weight 1)
    const uint16_t* regs;
    int region;
    uint32_t wsame, wdiff;
    int selfx;
    // point masks (batched counts): bit i of word i / 32 set = sorted point i
    // excluded; nullptr = no mask
    const uint32_t* mbA;
    const uint32_t* mbB;
    // point weights of two pixel maps (sorted order): each pair adds
    // wA[i] * wB[j]; nullptr for unweighted catalogs
    const uint32_t* wA;
    const uint32_t* wB;
    // radial pairs (M_RADIAL): redshifts in sorted order and the chord^2 of
    // the aperture; T1 then holds the unsquared redshift-difference edges
    const double* rA;
    const double* rB;
    double ap2;
    // the FP64 top threshold: a pair with d2 >= top64 is never counted
    // (T1[n1] for MONO, RMU and THETA; ap2 for radial pairs; for SIGMAPI
    // (sigma_max^2 + pi_max^2)(1 + 1e-12), rounded up)
    double top64;
    // the FP32 counterpart: d2_32 >= skip32 implies d2 >= top64 for the
    // canonical value (out_hi, or its SIGMAPI analogue)
    float skip32;
};

// A batched launch: the items (one CountArgs each, in device memory) share
// the binning whose tables are given here.
struct BatchArgs {
    const CountArgs* items;
    const uint32_t* chunks;         // per chunk: item, first tile, end tile, 0
    uint32_t nchunks;
    uint32_t* head;                 // next chunk to pop (global counter)
    int n1, n2, nbins, copies, hist_words;
    const double* T1;
    const double* T2;
    const float2* band1;
    const float2* band2;
};

// Host-side grid object.
struct GridHost {
    int device;
    cute_geometry geom;
    int64_t n;
    double L;
    int nx, ny, nz;
    double ox, oy, oz, ax, ay, az;
    double cx, cy, cz;
    double ext;          // max |x - c| over points and axes (FP32 rounding scale)
    double rawmax;       // max |raw coordinate|
    double lmax;         // max |p| over points (for |p + q| bounds)
    float4* p32;
    P64* p64;
    uint32_t* cstart;
    void* block;         // the one device allocation holding p64, p32 and cstart
    int tile_max;        // most points in a home tile (1..64)
    bool tile_auto;      // tile_max is the default (counts may cut tiles shorter)
    // pixel maps: occupancy of each point in sorted order, and the non-empty
    // pixels (ids ascending) with their occupancies, all in one allocation
    uint32_t* wt;        // nullptr for plain catalogs
    uint32_t* pix_id;
    uint32_t* pix_n;
    void* wblock;
    int n_cth, n_phi;
    // the build's start and end on its stream: work that uses the grid on any
    // stream waits for ev_ready on the device; the build time is read from
    // the pair when asked (nullptr when the build finished before returning)
    hipEvent_t ev_start, ev_ready;
    double ms_build;     // the build time when known without a wait (< 0: ask the events)
    GridView view() const;
};

// Make later work on stream s wait (on the device) for the build of g.
cute_status grid_wait(const cute_grid* g, hipStream_t s);

// Inputs of the FP32 rounding-error bounds (absolute errors per component).
struct ErrModel {
    double ec = 0.0;     // FP32 separation components
    double ec64 = 0.0;   // canonical FP64 separation components
    double el = 0.0;     // FP32 line-of-sight components (midpoint)
    double el64 = 0.0;   // FP64 line-of-sight components, before the sqrt(3) factor
};

// What one pair of grids contributes to a launch.
struct ItemGeom {
    GridView A, B;
    int geom = 0, is_auto = 0, periodic = 0;
    double L = 0.0, Rs = 0.0, th_s = 0.0, sin_th_s = 0.0;
    float offx = 0.f, offy = 0.f, offz = 0.f, lcx = 0.f, lcy = 0.f, lcz = 0.f;
    int max_w = 1;       // home-tile width limit in cells
    ErrModel em;
    double cost = 0.0;   // estimated candidate pairs
    // rows of neighbour cells as offsets from the home row (3-D grids of one
    // geometry): (dy, dz, cells left of c0, cells right of c1); empty when
    // the kernel must derive the rows itself
    std::vector<int4> stencil;
};

// A count launch: thresholds, band tables and the binning's kernel constants.
// number of floats cute_fp32_decision_tables writes to consts
constexpr int kDecisionConsts = 17;

struct Plan {
    int mode = 0, est = 0;
    double rmax = 0.0;               // largest countable separation
    std::vector<double> T1, T2;      // canonical thresholds
    std::vector<float2> band1, band2;
    CountArgs a;
    size_t lds = 0;                  // dynamic LDS bytes per workgroup
};

cute_status validate_binning(const cute_binning* b);
bool same_binning(const cute_binning* a, const cute_binning* b);
void plan_binning(const cute_binning* b, Plan& pl);
cute_status plan_item(const GridHost& A, const GridHost& B, bool is_auto, const cute_binning* b,
                      const Plan& pl, ItemGeom* g);
ErrModel max_err(const ErrModel& x, const ErrModel& y);
void plan_bands(const cute_binning* b, const ErrModel& em, Plan& pl);
cute_status plan_lds(Plan& pl, size_t extra);
void apply_item(const ItemGeom& g, CountArgs* a);
cute_status hip_status(hipError_t e, const char* what);

// error reporting
void set_error(const std::string& msg);
cute_status fail(cute_status s, const std::string& msg);

// exclusive scan of n uint32 values on the device (in may equal out)
cute_status exclusive_scan(const uint32_t* in, uint32_t* out, size_t n, hipStream_t s);

// home tiles of grid g (runs of <= 64 points in one row, x-extent <= max_w
// cells); *tiles is a stream-ordered allocation owned by the caller
// (reg: optional sorted-order region per point; tiles then never mix regions)
cute_status build_tiles(const GridHost& g, int max_w, hipStream_t s, Tile** tiles,
                        uint32_t* ntiles, const uint16_t* reg = nullptr);

// The same tiles without a wait for their count (no region labels): *tiles
// holds *cap = tile_count_bound slots, rows in order, with empty tiles
// (start == end) in the unused slots, for order_tiles to drop. *overflow
// (device memory) is raised if a row had more tiles than its slots.
class DevArena;
cute_status build_tiles_nowait(const GridHost& g, int max_w, hipStream_t s, Tile** tiles,
                               uint32_t* cap, uint32_t* overflow, DevArena* ar = nullptr);
// upper bound of the number of tiles of g (no region labels)
uint64_t tile_count_bound(const GridHost& g, int max_w);

// reorder *tiles longest first by estimated cost (needs the precomputed
// neighbour rows on the device; a no-op without them). With total set, empty
// tiles are dropped and the number kept is written to *total (device
// memory); without neighbour rows the kept tiles are then in no particular
// order. With ar, the temporaries and the new list come from the arena and
// the old list is not freed; otherwise the old list is freed and replaced.
cute_status order_tiles(const GridHost& A, const GridHost& B, const int4* stencil, int nst,
                        bool is_auto, bool periodic, Tile** tiles, uint32_t ntiles,
                        hipStream_t s, uint32_t* total = nullptr, DevArena* ar = nullptr);

// persistent count launch; *grid_used receives the number of workgroups
// out[i] = in[input index of sorted point i] for the n points of g (in:
// host or device memory); waits for the stream; rejects non-finite values.
cute_status gather_values(const GridHost& g, const double* in, bool on_device, double* out,
                          hipStream_t s);

// Add the pairs of objects that share a pixel of a pixel map to *bin.
cute_status add_pixel_self_pairs(const GridHost& g, unsigned long long* bin, hipStream_t s);

// A caller-provided device area for every temporary of a count, and two
// timing events made beforehand (the no-allocation entry point).
struct FixedArea {
    unsigned char* base;
    size_t cap;
    hipEvent_t events[2];
};

// The pair count of cute_count_pairs with all its device temporaries in
// *fixed (see there); counts and statistics as cute_count_pairs.
cute_status count_pairs_fixed(const cute_grid* a, const cute_grid* b, const cute_binning* bins,
                              cute_precision prec, uint64_t* counts, int32_t counts_on_device,
                              cute_count_stats* st, void* stream, const FixedArea* fixed);

cute_status launch_count(const CountArgs& args, int mode, int prec, int est, int wg_waves,
                         size_t lds_bytes, hipStream_t stream, int* grid_used);

// batched counts: kernel attributes and occupancy (not capturable), the
// launch itself (capturable), sorted-order mask bits, and a zero fill
cute_status batch_prepare(int mode, int prec, int est, size_t lds, int* per_cu);
cute_status batch_launch(const BatchArgs& ba, int mode, int prec, int est, int grid, size_t lds,
                         hipStream_t s);
cute_status mask_bits(const uint8_t* mask, const GridHost& g, uint32_t* bits, hipStream_t s);
cute_status zero_u64(unsigned long long* p, size_t n, hipStream_t s);
cute_status zero_u32(uint32_t* p, size_t n, hipStream_t s);

}  // namespace cute

struct cute_grid {
    cute::GridHost h;
};
