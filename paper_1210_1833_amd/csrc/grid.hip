// Cell-list ("chaining mesh") construction of Sec. 3.3: cubical cells over a
// box, or pixels of constant (cos theta, phi) extent on the sphere; points are
// counting-sorted by cell so that every row of cells is one contiguous run.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cute_internal.h"
#include "runtime.h"

namespace cute {

namespace {

constexpr int kBlock = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Per-block partial statistics of the raw input.
struct InStats {
    double lo[3], hi[3];
    double maxnorm2;      // max |p|^2
    unsigned long long bad_finite, bad_range, bad_unit;
};

__device__ inline void stats_init(InStats& s) {
    for (int d = 0; d < 3; d++) {
        s.lo[d] = INFINITY;
        s.hi[d] = -INFINITY;
    }
    s.maxnorm2 = 0.0;
    s.bad_finite = s.bad_range = s.bad_unit = 0;
}

__device__ inline void stats_merge(InStats& a, const InStats& b) {
    for (int d = 0; d < 3; d++) {
        a.lo[d] = fmin(a.lo[d], b.lo[d]);
        a.hi[d] = fmax(a.hi[d], b.hi[d]);
    }
    a.maxnorm2 = fmax(a.maxnorm2, b.maxnorm2);
    a.bad_finite += b.bad_finite;
    a.bad_range += b.bad_range;
    a.bad_unit += b.bad_unit;
}

__device__ void block_reduce_stats(InStats& s) {
    __shared__ InStats sh[kBlock];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) stats_merge(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    s = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_input_stats(const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ z, int64_t n,
                                                        int geom, double L, InStats* part) {
    InStats s;
    stats_init(s);
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double v[3] = {x[i], y[i], z[i]};
        bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
        if (!fin) {
            s.bad_finite++;
            continue;
        }
        for (int d = 0; d < 3; d++) {
            s.lo[d] = fmin(s.lo[d], v[d]);
            s.hi[d] = fmax(s.hi[d], v[d]);
        }
        double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        s.maxnorm2 = fmax(s.maxnorm2, n2);
        if (geom == CUTE_GEOM_BOX_PERIODIC) {
            for (int d = 0; d < 3; d++)
                if (!(v[d] >= 0.0 && v[d] < L)) {
                    s.bad_range++;
                    break;
                }
        } else if (geom == CUTE_GEOM_SPHERE) {
            if (fabs(n2 - 1.0) > 1e-6) s.bad_unit++;
        }
    }
    block_reduce_stats(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_stats_final(InStats* part, int nparts) {
    InStats s;
    stats_init(s);
    for (int i = threadIdx.x; i < nparts; i += kBlock) stats_merge(s, part[i]);
    block_reduce_stats(s);
    if (threadIdx.x == 0) part[0] = s;
}

struct CellGeo {
    int geom, nx, ny, nz;
    double ox, oy, oz, ax, ay, az, L;
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline uint32_t cell_of(const CellGeo& g, double x, double y, double z) {
    int ix, iy, iz;
    if (g.geom == CUTE_GEOM_SPHERE) {
        double phi = atan2(y, x);
        if (phi < 0.0) phi += kTwoPi;
        ix = clampi((int)floor(phi / g.ax), 0, g.nx - 1);
        iy = clampi((int)floor((z - g.oy) / g.ay), 0, g.ny - 1);
        iz = 0;
    } else {
        ix = clampi((int)floor((x - g.ox) / g.ax), 0, g.nx - 1);
        iy = clampi((int)floor((y - g.oy) / g.ay), 0, g.ny - 1);
        iz = clampi((int)floor((z - g.oz) / g.az), 0, g.nz - 1);
    }
    return (uint32_t)ix + (uint32_t)g.nx * ((uint32_t)iy + (uint32_t)g.ny * (uint32_t)iz);
}

// Points per thread of the key and scatter kernels: kPer independent loads
// and atomics per thread keep more of them in flight.
constexpr int kPer = 4;

// The rank of a point in its cell comes from a returning atomic on the cell's
// counter. Clustered catalogs put many points in a few cells, and atomics on
// one address serialise in L2, so a block first counts its own points per
// cell in an LDS table (open addressing, twice as many slots as points, so
// that probing always ends) and then takes one global atomic per distinct
// cell for the base of its ranks.
constexpr int kSlotBits = 11;
constexpr int kSlots = 1 << kSlotBits;
static_assert(kSlots >= 2 * kBlock * kPer, "the cell table must stay at most half full");
static_assert(kSlots % kBlock == 0, "whole slots per thread");
constexpr uint32_t kNoCell = 0xffffffffu;   // never a cell index (fewer than 2^26 cells)

__global__ __launch_bounds__(kBlock) void k_cell_keys(const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z, int64_t n,
                                                      CellGeo g, uint32_t* __restrict__ key,
                                                      uint32_t* __restrict__ rank,
                                                      uint32_t* __restrict__ count) {
    __shared__ uint32_t tcell[kSlots];
    __shared__ uint32_t tnum[kSlots];
    for (int j = threadIdx.x; j < kSlots; j += kBlock) {
        tcell[j] = kNoCell;
        tnum[j] = 0u;
    }
    const int64_t base = (int64_t)blockIdx.x * (kBlock * kPer) + threadIdx.x;
    uint32_t c[kPer], slot[kPer], local[kPer];
    double px[kPer], py[kPer], pz[kPer];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        // every load issued before the first use (a point past the end reads
        // the last one, n > 0, and is dropped)
        int64_t i = base + (int64_t)k * kBlock;
        i = i < n ? i : n - 1;
        px[k] = x[i];
        py[k] = y[i];
        pz[k] = z[i];
    }
#pragma unroll
    for (int k = 0; k < kPer; k++)
        c[k] = base + (int64_t)k * kBlock < n ? cell_of(g, px[k], py[k], pz[k]) : kNoCell;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        slot[k] = 0u;
        local[k] = 0u;
        if (c[k] == kNoCell) continue;
        uint32_t h = (c[k] * 2654435761u) >> (32 - kSlotBits);
        for (;;) {
            const uint32_t old = atomicCAS(&tcell[h], kNoCell, c[k]);
            if (old == kNoCell || old == c[k]) break;
            h = (h + 1u) & (kSlots - 1);
        }
        slot[k] = h;
        local[k] = atomicAdd(&tnum[h], 1u);
    }
    __syncthreads();
    {
        // one global atomic per distinct cell, all of a thread's in flight
        // together; tnum then holds the block's base rank in each cell
        constexpr int kSlotsPer = kSlots / kBlock;
        uint32_t m[kSlotsPer], cc[kSlotsPer];
#pragma unroll
        for (int q = 0; q < kSlotsPer; q++) {
            m[q] = tnum[threadIdx.x + q * kBlock];
            cc[q] = tcell[threadIdx.x + q * kBlock];
        }
#pragma unroll
        for (int q = 0; q < kSlotsPer; q++)
            if (m[q]) m[q] = atomicAdd(&count[cc[q]], m[q]);
#pragma unroll
        for (int q = 0; q < kSlotsPer; q++) tnum[threadIdx.x + q * kBlock] = m[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < n) {
            key[i] = c[k];
            rank[i] = tnum[slot[k]] + local[k];
        }
    }
}

// Exclusive scan, three phases: per-block scan of kScanItems items, scan of
// the block totals (recursively), then add the scanned totals back.
constexpr int kScanPer = 8;
constexpr int kScanItems = kBlock * kScanPer;

__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t sh[kBlock];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        uint32_t t = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t incl = sh[threadIdx.x];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_blocks(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, size_t n,
                                                        uint32_t* __restrict__ block_tot) {
    size_t base = (size_t)blockIdx.x * kScanItems + (size_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
    for (int k = 0; k < kScanPer; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan(s, &tot);
    for (int k = 0; k < kScanPer; k++) {
        if (base + k < n) out[base + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t* __restrict__ out, size_t n,
                                                     const uint32_t* __restrict__ block_pre) {
    size_t base = (size_t)blockIdx.x * kScanItems + (size_t)threadIdx.x * kScanPer;
    uint32_t add = block_pre[blockIdx.x];
    for (int k = 0; k < kScanPer; k++)
        if (base + k < n) out[base + k] += add;
}

__global__ __launch_bounds__(kBlock) void k_scatter(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    int64_t n, const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
    const uint32_t* __restrict__ cstart, double cx, double cy, double cz,
    float4* __restrict__ p32, P64* __restrict__ p64) {
    const int64_t base = (int64_t)blockIdx.x * (kBlock * kPer) + threadIdx.x;
    // all loads of the kPer points first, then the gathers of their cell
    // starts, then the stores (a point past the end reads the last one,
    // n > 0, and stores nothing)
    uint32_t kk[kPer], rk[kPer], pos[kPer];
    double a[kPer], b[kPer], c[kPer];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        int64_t i = base + (int64_t)k * kBlock;
        i = i < n ? i : n - 1;
        kk[k] = key[i];
        rk[k] = rank[i];
        a[k] = x[i];
        b[k] = y[i];
        c[k] = z[i];
    }
#pragma unroll
    for (int k = 0; k < kPer; k++) pos[k] = cstart[kk[k]] + rk[k];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i >= n) break;
        p32[pos[k]] = make_float4((float)(a[k] - cx), (float)(b[k] - cy), (float)(c[k] - cz), 0.0f);
        P64 q;
        q.x = a[k];
        q.y = b[k];
        q.z = c[k];
        q.idx = (uint32_t)i;
        q.pad = 0u;
        p64[pos[k]] = q;
    }
}

}  // namespace

// Exclusive scan of n uint32 values (in may equal out).
cute_status exclusive_scan(const uint32_t* in, uint32_t* out, size_t n, hipStream_t s) {
    if (n == 0) return CUTE_OK;
    size_t nb = (n + kScanItems - 1) / kScanItems;
    TempList tmp(s);
    uint32_t* tot = nullptr;
    cute_status st = tmp.alloc(&tot, nb);
    if (st != CUTE_OK) return st;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, tot);
    CUTE_HIP(hipGetLastError());
    if (nb > 1) {
        st = exclusive_scan(tot, tot, nb, s);
        if (st != CUTE_OK) return st;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, out, n, tot);
        CUTE_HIP(hipGetLastError());
    }
    return CUTE_OK;
}

GridView GridHost::view() const {
    GridView v;
    v.p32 = p32;
    v.p64 = p64;
    v.cstart = cstart;
    v.nx = nx;
    v.ny = ny;
    v.nz = nz;
    v.ox = ox;
    v.oy = oy;
    v.oz = oz;
    v.ax = ax;
    v.ay = ay;
    v.az = az;
    v.cx = cx;
    v.cy = cy;
    v.cz = cz;
    return v;
}

static constexpr int64_t kMaxCells = int64_t(1) << 26;
static constexpr int kMaxAxis = 65535;

// Choose the cells per axis and the cell geometry on the host.
static cute_status plan_cells(GridHost& g, const cute_grid_params* p, const InStats& s) {
    const int64_t n = g.n;
    double a = p->cell_size;
    if (g.geom == CUTE_GEOM_BOX_PERIODIC) {
        const double L = p->box_size;
        if (!(a > 0.0)) {
            double dens_a = std::cbrt(L * L * L / std::max<double>(1.0, (double)n) * 16.0);
            a = p->r_max > 0.0 ? std::max(p->r_max / 4.0, std::min(dens_a, p->r_max)) : dens_a;
        }
        int na = (int)std::max(1.0, std::floor(L / a));
        if (p->r_max > 0.0) {
            // a home tile one cell wide plus the stencil on both sides must not
            // wrap onto itself: 3 + 2 r_max / a <= cells per axis
            double f = 1.0 - 2.0 * p->r_max / L;
            int need = (int)std::ceil(3.0 / f) + 1;
            na = std::max(na, need);
        }
        while ((int64_t)na * na * na > kMaxCells) na--;
        na = std::min(na, 1024);
        g.nx = g.ny = g.nz = std::max(na, 1);
        g.ox = g.oy = g.oz = 0.0;
        g.ax = g.ay = g.az = L / g.nx;
        g.cx = g.cy = g.cz = 0.5 * L;
        g.ext = 0.5 * L;
        g.L = L;
    } else if (g.geom == CUTE_GEOM_BOX_OPEN) {
        double lo[3], hi[3], span = 0.0;
        for (int d = 0; d < 3; d++) {
            lo[d] = n ? s.lo[d] : 0.0;
            hi[d] = n ? s.hi[d] : 0.0;
            span = std::max(span, hi[d] - lo[d]);
        }
        if (!(a > 0.0)) {
            double vol = 1.0;
            for (int d = 0; d < 3; d++) vol *= std::max(hi[d] - lo[d], span * 1e-3 + 1e-300);
            double dens_a = std::cbrt(vol / std::max<double>(1.0, (double)n) * 16.0);
            a = p->r_max > 0.0 ? std::max(p->r_max / 4.0, std::min(dens_a, p->r_max)) : dens_a;
            if (!(a > 0.0)) a = 1.0;
        }
        int nd[3];
        for (;;) {
            int64_t tot = 1;
            for (int d = 0; d < 3; d++) {
                double c = std::ceil((hi[d] - lo[d]) / a);
                nd[d] = (int)std::min<double>(std::max(1.0, c), kMaxAxis);
                tot *= nd[d];
            }
            if (tot <= kMaxCells && nd[0] < kMaxAxis) break;
            a *= 1.25;
        }
        g.nx = nd[0];
        g.ny = nd[1];
        g.nz = nd[2];
        g.ox = lo[0];
        g.oy = lo[1];
        g.oz = lo[2];
        g.ax = g.ay = g.az = a;
        g.cx = 0.5 * (lo[0] + hi[0]);
        g.cy = 0.5 * (lo[1] + hi[1]);
        g.cz = 0.5 * (lo[2] + hi[2]);
        g.ext = 0.0;
        for (int d = 0; d < 3; d++) g.ext = std::max(g.ext, 0.5 * (hi[d] - lo[d]));
        g.ext *= 1.0 + 1e-12;
        g.L = 0.0;
    } else {  // SPHERE
        double zlo = n ? s.lo[2] : 0.0, zhi = n ? s.hi[2] : 0.0;
        if (!(a > 0.0)) {
            double area = kTwoPi * std::max(zhi - zlo, 1e-6);
            double dens_a = std::sqrt(area / std::max<double>(1.0, (double)n) * 16.0);
            a = p->r_max > 0.0 ? std::max(p->r_max / 4.0, std::min(dens_a, p->r_max)) : dens_a;
        }
        int nphi = (int)std::min<double>(std::max(1.0, std::floor(kTwoPi / a)), 8192);
        int nb = (int)std::min<double>(std::max(1.0, std::ceil((zhi - zlo) / a)), 8192);
        while ((int64_t)nphi * nb > kMaxCells) {
            nphi = std::max(1, nphi / 2);
            nb = std::max(1, nb / 2);
        }
        g.nx = nphi;
        g.ny = nb;
        g.nz = 1;
        g.ox = 0.0;
        g.oy = zlo;
        g.oz = 0.0;
        g.ax = kTwoPi / nphi;
        g.ay = (zhi > zlo) ? (zhi - zlo) / nb : 1.0;
        g.az = 1.0;
        g.cx = g.cy = g.cz = 0.0;
        g.ext = 1.0 + 1e-6;
        g.L = 0.0;
    }
    double rawmax = 0.0;
    for (int d = 0; d < 3; d++)
        rawmax = std::max(rawmax, std::max(std::fabs(n ? s.lo[d] : 0.0), std::fabs(n ? s.hi[d] : 0.0)));
    g.rawmax = rawmax;
    g.lmax = std::sqrt(s.maxnorm2) * (1.0 + 1e-12);
    return CUTE_OK;
}

}  // namespace cute

using namespace cute;

extern "C" cute_status cute_build_grid(const double* x, const double* y, const double* z,
                                       int64_t n, const cute_grid_params* p, void* stream,
                                       cute_grid** out) {
    if (!out) return fail(CUTE_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(CUTE_E_INVALID_ARG, "params is NULL");
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CUTE_E_INVALID_ARG, "n must be in [0, 2^31)");
    if (n > 0 && (!x || !y || !z)) return fail(CUTE_E_INVALID_ARG, "coordinate pointer is NULL");
    if (p->geom != CUTE_GEOM_BOX_PERIODIC && p->geom != CUTE_GEOM_BOX_OPEN &&
        p->geom != CUTE_GEOM_SPHERE)
        return fail(CUTE_E_INVALID_ARG, "unknown geometry");
    if (p->geom == CUTE_GEOM_BOX_PERIODIC && !(p->box_size > 0.0 && std::isfinite(p->box_size)))
        return fail(CUTE_E_INVALID_ARG, "periodic box needs a finite box_size > 0");
    if (!(p->cell_size >= 0.0) || !std::isfinite(p->cell_size))
        return fail(CUTE_E_INVALID_ARG, "cell_size must be >= 0");
    if (!(p->r_max >= 0.0) || !std::isfinite(p->r_max))
        return fail(CUTE_E_INVALID_ARG, "r_max must be >= 0");
    if (p->geom == CUTE_GEOM_BOX_PERIODIC && p->r_max >= 0.5 * p->box_size)
        return fail(CUTE_E_INVALID_ARG, "periodic r_max must be < L/2");
    if (p->tile_points < 0 || p->tile_points > 64)
        return fail(CUTE_E_INVALID_ARG, "tile_points must be in [0, 64]");

    int dev = 0;
    cute_status st = ensure_device_ready(&dev);
    if (st != CUTE_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    GridHost g;
    memset(&g, 0, sizeof(g));
    g.device = dev;
    g.geom = p->geom;
    g.n = n;
    g.tile_max = p->tile_points > 0 ? p->tile_points : 64;
    g.tile_auto = p->tile_points == 0;

    EventTimer timer(s);
    TempList tmp(s);
    const double *dx = x, *dy = y, *dz = z;
    if (!p->device_ptrs && n > 0) {
        double *hx, *hy, *hz;
        if ((st = tmp.alloc(&hx, n)) != CUTE_OK) return st;
        if ((st = tmp.alloc(&hy, n)) != CUTE_OK) return st;
        if ((st = tmp.alloc(&hz, n)) != CUTE_OK) return st;
        CUTE_HIP(hipMemcpyAsync(hx, x, n * sizeof(double), hipMemcpyHostToDevice, s));
        CUTE_HIP(hipMemcpyAsync(hy, y, n * sizeof(double), hipMemcpyHostToDevice, s));
        CUTE_HIP(hipMemcpyAsync(hz, z, n * sizeof(double), hipMemcpyHostToDevice, s));
        dx = hx;
        dy = hy;
        dz = hz;
    }

    // input statistics and validation (on the device, one small read-back)
    InStats stats;
    {
        int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
        InStats* part;
        if ((st = tmp.alloc(&part, nparts)) != CUTE_OK) return st;
        hipLaunchKernelGGL(k_input_stats, dim3(nparts), dim3(kBlock), 0, s, dx, dy, dz, n,
                           (int)p->geom, p->box_size, part);
        CUTE_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kBlock), 0, s, part, nparts);
        CUTE_HIP(hipGetLastError());
        CUTE_HIP(hipMemcpyAsync(&stats, part, sizeof(InStats), hipMemcpyDeviceToHost, s));
        CUTE_HIP(hipStreamSynchronize(s));
    }
    if (stats.bad_finite) return fail(CUTE_E_INVALID_ARG, "non-finite coordinates");
    if (stats.bad_range) return fail(CUTE_E_INVALID_ARG, "periodic coordinates outside [0, L)");
    if (stats.bad_unit) return fail(CUTE_E_INVALID_ARG, "SPHERE needs unit vectors");

    if ((st = plan_cells(g, p, stats)) != CUTE_OK) return st;
    const int64_t ncells = (int64_t)g.nx * g.ny * g.nz;

    cute_grid* grid = new (std::nothrow) cute_grid;
    if (!grid) return fail(CUTE_E_OUT_OF_MEMORY, "host allocation");
    auto cleanup = [&](cute_status e) {
        dfree(g.block, s);
        delete grid;
        return e;
    };
    // one block per grid: [p64 (32 B per point) | p32 (16 B) | cstart]
    unsigned char* blk = nullptr;
    const size_t b64 = (size_t)n * sizeof(P64), b32 = (size_t)n * sizeof(float4);
    if ((st = dalloc(&blk, b64 + b32 + ((size_t)ncells + 1) * sizeof(uint32_t), s)) != CUTE_OK)
        return cleanup(st);
    g.block = blk;
    g.p64 = reinterpret_cast<P64*>(blk);
    g.p32 = reinterpret_cast<float4*>(blk + b64);
    g.cstart = reinterpret_cast<uint32_t*>(blk + b64 + b32);

    uint32_t* key = nullptr;  // keys and ranks in one temporary
    if ((st = tmp.alloc(&key, 2 * (size_t)n)) != CUTE_OK) return cleanup(st);
    uint32_t* rank = key + n;
    if ((st = zero_u32(g.cstart, (size_t)ncells + 1, s)) != CUTE_OK) return cleanup(st);
    CellGeo cg{(int)g.geom, g.nx, g.ny, g.nz, g.ox, g.oy, g.oz, g.ax, g.ay, g.az, g.L};
    if (n > 0) {
        unsigned nb = (unsigned)((n + kBlock * kPer - 1) / (kBlock * kPer));
        hipLaunchKernelGGL(k_cell_keys, dim3(nb), dim3(kBlock), 0, s, dx, dy, dz, n, cg, key, rank,
                           g.cstart);
        if (hipGetLastError() != hipSuccess) return cleanup(fail(CUTE_E_DEVICE, "cell keys launch"));
    }
    if ((st = exclusive_scan(g.cstart, g.cstart, (size_t)ncells + 1, s)) != CUTE_OK)
        return cleanup(st);
    if (n > 0) {
        unsigned nb = (unsigned)((n + kBlock * kPer - 1) / (kBlock * kPer));
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, s, dx, dy, dz, n, key, rank,
                           g.cstart, g.cx, g.cy, g.cz, g.p32, g.p64);
        if (hipGetLastError() != hipSuccess) return cleanup(fail(CUTE_E_DEVICE, "scatter launch"));
    }
    // the end event follows the last kernel; the grid keeps both events, and
    // work that uses it (on any stream) waits for the end on the device, so
    // the call returns without waiting (the host inputs were copied before
    // the statistics read-back above)
    timer.stop();
    if (timer.a && timer.b) {
        g.ev_start = timer.a;
        g.ev_ready = timer.b;
        timer.a = timer.b = nullptr;   // owned by the grid from here on
        g.ms_build = -1.0;
    } else {
        if (hipStreamSynchronize(s) != hipSuccess) return cleanup(fail(CUTE_E_DEVICE, "build sync"));
        g.ms_build = 0.0;
    }
    grid->h = g;
    *out = grid;
    return CUTE_OK;
}

cute_status cute::grid_wait(const cute_grid* g, hipStream_t s) {
    if (g && g->h.ev_ready) CUTE_HIP(hipStreamWaitEvent(s, g->h.ev_ready, 0));
    return CUTE_OK;
}

extern "C" void cute_free_grid(cute_grid* g) {
    if (!g) return;
    // the buffers come from the stream-ordered pool; the caller guarantees
    // that no work on any stream still uses the grid, and the build itself is
    // waited for (in practice long finished: any count of the grid returned)
    if (g->h.ev_ready) {
        (void)hipEventSynchronize(g->h.ev_ready);
        (void)hipEventDestroy(g->h.ev_ready);
    }
    if (g->h.ev_start) (void)hipEventDestroy(g->h.ev_start);
    dfree(g->h.block, nullptr);
    dfree(g->h.wblock, nullptr);
    delete g;
}

extern "C" cute_status cute_get_grid_info(const cute_grid* g, cute_grid_info* info) {
    if (!g || !info) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    info->n = g->h.n;
    info->dims[0] = g->h.nx;
    info->dims[1] = g->h.ny;
    info->dims[2] = g->h.nz;
    info->cell[0] = g->h.ax;
    info->cell[1] = g->h.ay;
    info->cell[2] = g->h.az;
    info->origin[0] = g->h.ox;
    info->origin[1] = g->h.oy;
    info->origin[2] = g->h.oz;
    info->ms_build = g->h.ms_build;
    if (g->h.ev_ready) {
        // the build time: wait for its end event
        CUTE_HIP(hipEventSynchronize(g->h.ev_ready));
        float ms = 0.f;
        if (g->h.ev_start) CUTE_HIP(hipEventElapsedTime(&ms, g->h.ev_start, g->h.ev_ready));
        info->ms_build = ms;
    }
    return CUTE_OK;
}
