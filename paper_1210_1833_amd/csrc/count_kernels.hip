// Pair-count kernels for gfx950.
//
// One wavefront owns one home tile at a time (a run of up to 64 sorted points
// inside one row of cells) and walks the neighbour cells of Sec. 3.3 as
// contiguous spans of the other catalog. The spans are cut into chunks of 64
// neighbour points, one per lane in VGPRs; the home points are wave-uniform
// and arrive four at a time through scalar loads, so that each lane evaluates
// four independent pairs per step. Counts go to one 64-bit LDS histogram per
// workgroup (several interleaved copies, so that lanes hitting the same bin
// use different banks), summed into uint64 global counts at the end.
//
// Precision paths
//  - FP64: every pair is classified by the canonical FP64 predicates.
//  - FP32_EDGE: separations in FP32; a pair is counted directly only when its
//    FP32 value is farther than a proven rounding bound from every decision
//    threshold (bin edges, r_max, mu edges); the rest go to a per-wave LDS
//    queue that is drained 64 pairs at a time through the canonical FP64
//    predicates, so the counts equal the FP64 ones.
//  - FP32_ONLY: FP32 decisions only.
#include <map>
#include <mutex>
#include <tuple>

#include "count_device.h"

namespace cute {

namespace {

// Four 4-wave workgroups per CU: the register budget stays at 128 VGPRs.
// The one-variable FP32_EDGE kernels (MONO, THETA) run five (96 VGPRs),
// which hides more latency: the angular count takes 10 % less time; the r-mu
// and sigma-pi ones gain nothing.
// WT: pixel maps, each pair weighted by the product of the point weights.
template <int MODE, int PREC, int EST, bool WT>
__global__ __launch_bounds__(256, (kWgPerCu<MODE, PREC>)) void k_count(CountArgs P) {
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
    constexpr bool H32 = kH32<MODE>;
    // the histogram: hist_words counters of 4 (kH32) or 8 bytes, padded to 8
    unsigned char* hist0 = reinterpret_cast<unsigned char*>(B2 + (n2p > 0 ? n2p : 1));
    const size_t hbytes = ((size_t)P.hist_words * (H32 ? 4 : 8) + 7) & ~(size_t)7;
    uint32_t* q0 = reinterpret_cast<uint32_t*>(hist0 + hbytes);
    unsigned long long* rs0 = reinterpret_cast<unsigned long long*>(q0 + (size_t)nwaves * 3 * kQCap);
    uint32_t* sp0 = reinterpret_cast<uint32_t*>(rs0 + 2 * nwaves);
    uint32_t* budget = sp0 + (size_t)nwaves * 3 * kSpanCap;  // 32-bit histograms only
    for (int i = threadIdx.x; i <= n1; i += blockDim.x) T1[i] = P.T1[i];
    for (int i = threadIdx.x; i <= n2p; i += blockDim.x) T2[i] = n2p ? P.T2[i] : 0.0;
    if (PREC != P_FP64) {
        for (int i = threadIdx.x; i < n1; i += blockDim.x) B1[i] = P.band1[i];
        for (int i = threadIdx.x; i < n2p; i += blockDim.x) B2[i] = P.band2[i];
    }
    for (size_t i = threadIdx.x; i < hbytes / 4; i += blockDim.x) reinterpret_cast<uint32_t*>(hist0)[i] = 0u;
    for (int i = threadIdx.x; i < 2 * nwaves; i += blockDim.x) rs0[i] = 0ull;
    if (H32 && threadIdx.x == 0) *budget = 0u;
    __syncthreads();

    WaveState W;
    W.hist = hist0;
    W.budget = budget;
    W.pend = 0;
    W.qi = q0 + (size_t)wave * 3 * kQCap;
    W.qj = W.qi + kQCap;
    W.qc = W.qj + kQCap;
    W.rstat = rs0 + 2 * wave;
    W.tail = 0;
    W.evals = W.tiles = 0;
    SpanBuf S;
    S.a = sp0 + (size_t)wave * 3 * kSpanCap;
    S.b = S.a + kSpanCap;
    S.f = S.b + kSpanCap;
    S.n = 0;

    const uint32_t ntiles = P.ntiles_dev ? uni(*P.ntiles_dev) : P.ntiles;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(P.work_head, 1u);
        t = uni(t);
        if (t >= ntiles) break;
        const cu32p tp = (cu32p)(const void*)P.tiles;
        Tile tl;
        tl.start = uni(tp[4 * t]);
        tl.end = uni(tp[4 * t + 1]);
        tl.row = uni(tp[4 * t + 2]);
        tl.c0c1 = uni(tp[4 * t + 3]);
        do_tile<MODE, PREC, EST, false, WT>(P, W, S, B1, B2, T1, T2, lane, tl);
    }
    if constexpr (PREC == P_FP32E)
        W.tail = drain_queue<MODE, EST>(P.self, W.hist, W.qi, W.qj, W.qc, W.rstat, B1, B2, T1, T2, lane,
                                        W.tail, true);
    if (lane == 0) {
        atomicAdd(&P.stats[0], (unsigned long long)W.evals);
        atomicAdd(&P.stats[1], W.rstat[0]);
        atomicAdd(&P.stats[2], W.rstat[1]);
        atomicAdd(&P.stats[3], (unsigned long long)W.tiles);
    }
    __syncthreads();
    // sum the copies, then one global atomic per non-empty bin
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) {
        uint64_t s = 0;
        if constexpr (H32) {
            const uint32_t* hh = reinterpret_cast<const uint32_t*>(hist0) + (size_t)b * P.copies;
            for (int c = 0; c < P.copies; c++) s += hh[c];
        } else {
            const unsigned long long* hh = reinterpret_cast<const unsigned long long*>(hist0) + (size_t)b * P.copies;
            for (int c = 0; c < P.copies; c++) s += hh[c];
        }
        if (s) atomicAdd(&P.counts[b], (unsigned long long)s);
    }
}

template <int MODE, int PREC, int EST, bool WT>
cute_status launch_one(const CountArgs& a, int wg_waves, size_t lds, hipStream_t s, int* grid_used) {
    auto kern = k_count<MODE, PREC, EST, WT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_status(e, "hipFuncSetAttribute");
    }
    // occupancy of this variant at this LDS size, queried once per device
    static std::mutex mu;
    static std::map<std::tuple<int, int, size_t, bool>, std::pair<int, int>> cache;
    int dev = 0, ncu = 0, per_cu = 0;
    CUTE_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(std::make_tuple(dev, wg_waves, lds, WT));
        if (it != cache.end()) {
            ncu = it->second.first;
            per_cu = it->second.second;
        }
    }
    if (ncu == 0) {
        CUTE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        CUTE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wg_waves, lds));
        if (per_cu < 1) per_cu = 1;
        std::lock_guard<std::mutex> lk(mu);
        cache[std::make_tuple(dev, wg_waves, lds, WT)] = std::make_pair(ncu, per_cu);
    }
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
    if (a.wA != nullptr) {
        // weighted pairs: the angular kernels only (pixel maps)
        if constexpr (MODE == M_THETA) {
            if (est_log(est)) return launch_one<MODE, PREC, E_LOG, true>(a, wg_waves, lds, s, g);
            return launch_one<MODE, PREC, E_LIN, true>(a, wg_waves, lds, s, g);
        } else {
            return fail(CUTE_E_UNSUPPORTED, "weighted pairs need a THETA binning");
        }
    }
    if constexpr (MODE == M_RMU_Z && PREC == P_FP32E) {
        // the mu decision in mu space (FP32_EDGE only)
        if (est == (E_LOG | E_MUF)) return launch_one<MODE, PREC, E_LOG | E_MUF, false>(a, wg_waves, lds, s, g);
        if (est == E_MUF) return launch_one<MODE, PREC, E_MUF, false>(a, wg_waves, lds, s, g);
    }
    if (est_log(est)) return launch_one<MODE, PREC, E_LOG, false>(a, wg_waves, lds, s, g);
    return launch_one<MODE, PREC, E_LIN, false>(a, wg_waves, lds, s, g);
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
        case M_RADIAL:
            // few pairs fall inside an aperture: FP64 only
            if (prec != P_FP64 || args.wA != nullptr)
                return fail(CUTE_E_UNSUPPORTED, "radial counts are FP64 and unweighted");
            return launch_one<M_RADIAL, P_FP64, E_LIN, false>(args, wg_waves, lds_bytes, stream, grid_used);
        default: return fail(CUTE_E_INTERNAL, "unknown mode");
    }
}

// Home tiles: each row of cells is cut into runs of at most tmax points
// whose x-extent stays within max_w cells (so that periodic stencils never
// wrap onto themselves); a cell with more points is split. With a region per
// point (points sorted by region inside each cell), a tile also ends where
// the region changes. One thread walks one row; with out == nullptr it only
// counts the tiles. Only the first cap tiles are written; the count returned
// includes any beyond.
__device__ uint32_t walk_row_tiles(const uint32_t* __restrict__ cstart, const uint16_t* __restrict__ reg,
                                   int nx, int r, int max_w, uint32_t tmax, Tile* __restrict__ out,
                                   uint32_t cap = 0xffffffffu) {
    const uint32_t* cs = cstart + (size_t)r * nx;
    uint32_t o = 0, fill = 0;
    int first = -1;
    uint16_t cur_rg = 0;
    Tile cur{0u, 0u, 0u, 0u};
    bool open = false;
    // cell offsets in batches of eight (independent loads in flight); the
    // batch loop is unrolled so that the offsets stay in registers
    constexpr int kB = 8;
    for (int cb = 0; cb < nx; cb += kB) {
        uint32_t ofs[kB + 1];
#pragma unroll
        for (int i = 0; i <= kB; i++) ofs[i] = cb + i <= nx ? cs[cb + i] : 0u;
#pragma unroll
        for (int k = 0; k < kB; k++) {
            const int c = cb + k;
            if (c >= nx) break;
            uint32_t pos = ofs[k];
            const uint32_t end = ofs[k + 1];
            while (pos < end) {
                // the next run of points of one region inside this cell
                uint32_t run = end - pos;
                uint16_t rg = 0;
                if (reg != nullptr) {
                    rg = reg[pos];
                    run = 1;
                    while (pos + run < end && reg[pos + run] == rg) run++;
                }
                while (run > 0) {
                    if (!open || fill == tmax || c - first + 1 > max_w || rg != cur_rg) {
                        if (open) {
                            if (out && o < cap) out[o] = cur;
                            o++;
                        }
                        open = true;
                        fill = 0;
                        first = c;
                        cur_rg = rg;
                        cur.start = pos;
                        cur.end = pos;
                        cur.row = (uint32_t)r;
                        cur.c0c1 = (uint32_t)c | ((uint32_t)c << 16);
                    }
                    const uint32_t take = tmax - fill < run ? tmax - fill : run;
                    fill += take;
                    run -= take;
                    pos += take;
                    cur.end = pos;
                    cur.c0c1 = (cur.c0c1 & 0xffffu) | ((uint32_t)c << 16);
                }
            }
        }
    }
    if (open) {
        if (out && o < cap) out[o] = cur;
        o++;
    }
    return o;
}

__global__ __launch_bounds__(256) void k_tiles_count(const uint32_t* __restrict__ cstart,
                                                     const uint16_t* __restrict__ reg, int nx,
                                                     int nrows, int max_w, uint32_t tmax,
                                                     uint32_t* __restrict__ ntile) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) ntile[nrows] = 0u;  // the scan's last entry becomes the total
    if (r >= nrows) return;
    ntile[r] = walk_row_tiles(cstart, reg, nx, r, max_w, tmax, nullptr);
}

__global__ __launch_bounds__(256) void k_tiles_write(const uint32_t* __restrict__ cstart,
                                                     const uint16_t* __restrict__ reg, int nx,
                                                     int nrows, int max_w, uint32_t tmax,
                                                     const uint32_t* __restrict__ toff,
                                                     Tile* __restrict__ tiles,
                                                     uint32_t* __restrict__ total) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0 && total != nullptr) *total = toff[nrows];
    if (r >= nrows) return;
    (void)walk_row_tiles(cstart, reg, nx, r, max_w, tmax, tiles + toff[r]);
}

// Tiles without a count pass. Row r, whose points are [s_r, s_{r+1}), owns
// the slots from b_r = floor(s_r / tmax) + r (W + 1), W = floor((nx - 1) /
// max_w), up to b_{r+1}: the rows partition [0, tile_count_bound) exactly, so
// every slot is written, with a tile or as empty. A row of p points has at
// most floor(p / tmax) + W + 1 tiles (see tile_count_bound), which is at most
// b_{r+1} - b_r because floor(s / tmax) + floor(p / tmax) <= floor((s + p) /
// tmax). The last row also takes any slots left before cap, the length of
// out, and no row writes at or past cap. A row with more tiles than slots
// (the bound failing) raises *overflow.
// One wave per row: the lanes load 64 cell offsets at a time, the walk (the
// cuts of walk_row_tiles without regions, on wave-uniform values) reads them
// with readlane, lane 0 writes the tiles and all lanes the empty slots.
__global__ __launch_bounds__(256) void k_tiles_sparse(const uint32_t* __restrict__ cstart, int nx,
                                                      int nrows, int max_w, uint32_t tmax,
                                                      Tile* __restrict__ out, uint32_t cap,
                                                      uint32_t* __restrict__ overflow) {
    const int lane = (int)(threadIdx.x & 63u);
    const int r = unii((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (r >= nrows) return;
    const uint32_t* cs = cstart + (size_t)r * nx;
    const uint64_t W1 = (uint64_t)((uint32_t)(nx - 1) / (uint32_t)max_w) + 1u;
    const uint32_t p0 = uni(cs[0]), p1 = uni(cs[nx]);
    const uint64_t b0 = (uint64_t)(p0 / tmax) + (uint64_t)r * W1;
    uint64_t b1 = r + 1 == nrows ? (uint64_t)cap : (uint64_t)(p1 / tmax) + (uint64_t)(r + 1) * W1;
    bool over = false;
    if (b1 > cap) {
        over = true;
        b1 = cap;
    }
    const uint32_t slots = b0 < b1 ? (uint32_t)(b1 - b0) : 0u;
    Tile* o = out + b0;
    uint32_t k = 0, fill = 0;
    int first = -1;
    bool open = false;
    Tile cur{0u, 0u, 0u, 0u};
    for (int cb = 0; cb < nx; cb += 64) {
        // offsets of cells cb .. cb + 63 in the lanes, of cell cb + 64 beside
        const uint32_t v = cb + lane <= nx ? cs[cb + lane] : 0u;
        const uint32_t vn = cb + 64 <= nx ? uni(cs[cb + 64]) : 0u;
        const int m = nx - cb < 64 ? nx - cb : 64;
        for (int j = 0; j < m; j++) {
            const int c = cb + j;
            uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)v, j);
            const uint32_t end = j + 1 < 64 ? (uint32_t)__builtin_amdgcn_readlane((int)v, j + 1) : vn;
            while (pos < end) {
                if (!open || fill == tmax || c - first + 1 > max_w) {
                    if (open) {
                        if (lane == 0 && k < slots) o[k] = cur;
                        k++;
                    }
                    open = true;
                    fill = 0;
                    first = c;
                    cur.start = pos;
                    cur.end = pos;
                    cur.row = (uint32_t)r;
                    cur.c0c1 = (uint32_t)c | ((uint32_t)c << 16);
                }
                const uint32_t take = tmax - fill < end - pos ? tmax - fill : end - pos;
                fill += take;
                pos += take;
                cur.end = pos;
                cur.c0c1 = (cur.c0c1 & 0xffffu) | ((uint32_t)c << 16);
            }
        }
    }
    if (open) {
        if (lane == 0 && k < slots) o[k] = cur;
        k++;
    }
    if ((over || k > slots) && lane == 0) atomicOr(overflow, 1u);
    for (uint32_t i = k + (uint32_t)lane; i < slots; i += 64u) o[i] = Tile{0u, 0u, 0u, 0u};
}

namespace {

// Estimated cost of each home tile for the longest-first order: candidate
// pairs (home points times the neighbours its stencil rows hold) plus a
// per-row and a per-tile overhead, in pair evaluations. Uses the precomputed
// neighbour rows (grids of one geometry), so it is integer work.
constexpr uint32_t kCostBuckets = 256;

constexpr uint32_t kNoTile = 0xffffffffu;  // the key of an empty slot

// One wave per tile slot, the lanes taking the stencil rows; writes the
// tile's cost bucket to key[t] (kNoTile for an empty slot).
__global__ __launch_bounds__(256) void k_tile_cost(const Tile* __restrict__ tiles, uint32_t ntiles,
                                                   const uint32_t* __restrict__ cs, int any, int nx,
                                                   int ny, int nz, const int4* __restrict__ st,
                                                   int nst, int periodic, int is_auto,
                                                   uint32_t* __restrict__ key) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t t = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (t >= ntiles) return;
    const cu32p tp = (cu32p)(const void*)tiles;
    Tile tl;
    tl.start = uni(tp[4 * t]);
    tl.end = uni(tp[4 * t + 1]);
    tl.row = uni(tp[4 * t + 2]);
    tl.c0c1 = uni(tp[4 * t + 3]);
    if (tl.end <= tl.start) {  // empty slots are not tiles
        if (lane == 0) key[t] = kNoTile;
        return;
    }
    const int c0 = (int)(tl.c0c1 & 0xffffu), c1 = (int)(tl.c0c1 >> 16);
    const int cy = (int)(tl.row % (uint32_t)any), cz = (int)(tl.row / (uint32_t)any);
    uint64_t nb = 0;
    uint32_t rows = 0;
    for (int e = lane; e < nst; e += 64) {
        const int4 o = st[e];
        int by = cy + o.x, bz = cz + o.y;
        const bool same = is_auto && o.x == 0 && o.y == 0;
        int x0 = same ? c0 : c0 - o.z, x1 = c1 + o.w;
        if (periodic) {
            by -= floordiv(by, ny) * ny;
            bz -= floordiv(bz, nz) * nz;
            x1 = x1 < x0 + nx - 1 ? x1 : x0 + nx - 1;
        } else {
            if (by < 0 || by >= ny || bz < 0 || bz >= nz) continue;
            x0 = x0 < 0 ? 0 : x0;
            x1 = x1 > nx - 1 ? nx - 1 : x1;
            if (x0 > x1) continue;
        }
        const uint32_t rb = (uint32_t)nx * ((uint32_t)by + (uint32_t)ny * (uint32_t)bz);
        for (int a0 = x0; a0 <= x1;) {
            const int kx = floordiv(a0, nx);
            const int lim = (kx + 1) * nx - 1;
            const int a1 = x1 < lim ? x1 : lim;
            nb += cs[rb + (uint32_t)(a1 - kx * nx) + 1u] - cs[rb + (uint32_t)(a0 - kx * nx)];
            a0 = a1 + 1;
        }
        rows++;
    }
    for (int off = 32; off > 0; off >>= 1) {
        nb += __shfl_xor(nb, off);
        rows += __shfl_xor(rows, off);
    }
    if (lane == 0) {
        // bucket on a log scale, 8 per octave, largest cost first (bucket 0);
        // log2(c) is in [11, 64)
        const uint64_t c = (uint64_t)(tl.end - tl.start) * nb + 128ull * rows + 2048ull;
        const float lc = (__builtin_amdgcn_logf((float)c) - 11.0f) * 8.0f;
        key[t] = kCostBuckets - 1u - (uint32_t)fminf(fmaxf(lc, 0.0f), (float)(kCostBuckets - 1));
    }
}

// Compaction without a cost estimate (grids without precomputed neighbour
// rows): every tile gets bucket 0, an empty slot kNoTile.
__global__ __launch_bounds__(256) void k_tile_live(const Tile* __restrict__ tiles, uint32_t ntiles,
                                                   uint32_t* __restrict__ key) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    key[t] = tl.end > tl.start ? 0u : kNoTile;
}

// Rank of each tile within its bucket: LDS atomics inside the block, then one
// global atomic per (block, bucket) reserves the block's range. (A thread past
// the end or on an empty slot joins the barriers and counts nothing.)
__global__ __launch_bounds__(256) void k_tile_rank(const uint32_t* __restrict__ key, uint32_t ntiles,
                                                   uint32_t* __restrict__ rank,
                                                   uint32_t* __restrict__ hist) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t b = t < ntiles ? key[t] : kNoTile;
    const bool live = b != kNoTile;
    __shared__ uint32_t lh[kCostBuckets], lbase[kCostBuckets];
    for (uint32_t i = threadIdx.x; i < kCostBuckets; i += blockDim.x) lh[i] = 0u;
    __syncthreads();
    const uint32_t lr = live ? atomicAdd(&lh[b], 1u) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kCostBuckets; i += blockDim.x)
        if (lh[i]) lbase[i] = atomicAdd(&hist[i], lh[i]);
    __syncthreads();
    if (live) rank[t] = lbase[b] + lr;
}

// Scatter the tiles into bucket order: every block scans the bucket counts in
// LDS (kCostBuckets of them), then each tile goes to its bucket's offset plus
// its rank within the bucket.
__global__ __launch_bounds__(256) void k_tile_scatter(const Tile* __restrict__ tiles, uint32_t ntiles,
                                                      const uint32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ rank,
                                                      const uint32_t* __restrict__ hist,
                                                      Tile* __restrict__ out,
                                                      uint32_t* __restrict__ total) {
    __shared__ uint32_t off[kCostBuckets];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t b = 0; b < kCostBuckets; b++) {
            off[b] = acc;
            acc += hist[b];
        }
        if (blockIdx.x == 0 && total != nullptr) *total = acc;
    }
    __syncthreads();
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const uint32_t b = key[t];
    if (b == kNoTile) return;  // an empty slot
    out[off[b] + rank[t]] = tiles[t];
}

}  // namespace

// Reorder tiles longest first (estimated cost, descending): the persistent
// waves take the heavy tiles early and the light ones fill the tail. Without
// neighbour rows the tiles keep their order, unless total is set: then the
// empty slots are only dropped (tiles in no particular order).
cute_status order_tiles(const GridHost& A, const GridHost& B, const int4* stencil, int nst,
                        bool is_auto, bool periodic, Tile** tiles, uint32_t ntiles,
                        hipStream_t s, uint32_t* total, DevArena* ar) {
    const bool rows = stencil != nullptr && nst > 0;
    if (total != nullptr && ntiles == 0) return fail(CUTE_E_INTERNAL, "tile compaction without tiles");
    if (total == nullptr && (ntiles < 2 || !rows)) return CUTE_OK;
    DevArena pool(s);
    DevArena& mem = ar != nullptr ? *ar : pool;
    uint32_t *key = nullptr, *rank = nullptr, *hist = nullptr;
    Tile* t1 = nullptr;
    cute_status st;
    if ((st = mem.get(&key, ntiles)) != CUTE_OK) return st;
    if ((st = mem.get(&rank, ntiles)) != CUTE_OK) return st;
    if ((st = mem.get(&hist, kCostBuckets)) != CUTE_OK) return st;
    if ((st = zero_u32(hist, kCostBuckets, s)) != CUTE_OK) return st;
    // the reordered list outlives this call: from the caller's arena, or its
    // own pool allocation that replaces (and frees) the input list
    if (ar != nullptr) {
        if ((st = ar->get(&t1, ntiles)) != CUTE_OK) return st;
    } else if ((st = dalloc(&t1, ntiles, s)) != CUTE_OK) {
        return st;
    }
    const unsigned nb = (ntiles + 255u) / 256u;
    if (rows) {
        hipLaunchKernelGGL(k_tile_cost, dim3((ntiles + 3u) / 4u), dim3(256), 0, s, *tiles, ntiles,
                           B.cstart, A.ny, B.nx, B.ny, B.nz, stencil, nst, periodic ? 1 : 0,
                           is_auto ? 1 : 0, key);
    } else {
        hipLaunchKernelGGL(k_tile_live, dim3(nb), dim3(256), 0, s, *tiles, ntiles, key);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tile_rank, dim3(nb), dim3(256), 0, s, key, ntiles, rank, hist);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tile_scatter, dim3(nb), dim3(256), 0, s, *tiles, ntiles, key, rank,
                           hist, t1, total);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        if (ar == nullptr) dfree(t1, s);
        return hip_status(e, "tile order");
    }
    if (ar == nullptr) dfree(*tiles, s);
    *tiles = t1;
    return CUTE_OK;
}

cute_status build_tiles(const GridHost& g, int max_w, hipStream_t s, Tile** tiles,
                        uint32_t* ntiles, const uint16_t* reg) {
    *tiles = nullptr;
    *ntiles = 0;
    const int nrows = g.ny * g.nz;
    TempList tmp(s);
    uint32_t* cnt = nullptr;
    cute_status st = tmp.alloc(&cnt, (size_t)nrows + 1);
    if (st != CUTE_OK) return st;
    const unsigned nb = (unsigned)((nrows + 255) / 256);
    hipLaunchKernelGGL(k_tiles_count, dim3(nb), dim3(256), 0, s, g.cstart, reg, g.nx, nrows, max_w,
                       (uint32_t)g.tile_max, cnt);
    CUTE_HIP(hipGetLastError());
    if ((st = exclusive_scan(cnt, cnt, (size_t)nrows + 1, s)) != CUTE_OK) return st;
    uint32_t total = 0;
    CUTE_HIP(hipMemcpyAsync(&total, cnt + nrows, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CUTE_HIP(hipStreamSynchronize(s));
    Tile* t = nullptr;
    if ((st = dalloc(&t, total, s)) != CUTE_OK) return st;
    if (total > 0) {
        hipLaunchKernelGGL(k_tiles_write, dim3(nb), dim3(256), 0, s, g.cstart, reg, g.nx, nrows,
                           max_w, (uint32_t)g.tile_max, cnt, t, (uint32_t*)nullptr);
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

// In a row, a tile is opened by the row's first point, after a tile of tmax
// points (at most floor(points / tmax) times) or when the next point lies
// max_w cells or more past the open tile's first cell (the first cell then
// advances by at least max_w: at most floor((nx - 1) / max_w) times).
uint64_t tile_count_bound(const GridHost& g, int max_w) {
    const uint64_t rows = (uint64_t)g.ny * (uint64_t)g.nz;
    const uint64_t w = (uint64_t)(max_w < 1 ? 1 : max_w);
    return (uint64_t)g.n / (uint64_t)g.tile_max + rows * ((uint64_t)(g.nx - 1) / w + 1u);
}

cute_status build_tiles_nowait(const GridHost& g, int max_w, hipStream_t s, Tile** tiles,
                               uint32_t* cap, uint32_t* overflow, DevArena* ar) {
    *tiles = nullptr;
    *cap = 0;
    const uint64_t bound = tile_count_bound(g, max_w);
    if (bound >= (uint64_t(1) << 31)) return fail(CUTE_E_INTERNAL, "tile bound too large");
    const int nrows = g.ny * g.nz;
    Tile* t = nullptr;
    cute_status st = ar != nullptr ? ar->get(&t, (size_t)bound) : dalloc(&t, (size_t)bound, s);
    if (st != CUTE_OK) return st;
    const unsigned nb = (unsigned)((nrows + 3) / 4);  // one wave per row
    hipLaunchKernelGGL(k_tiles_sparse, dim3(nb), dim3(256), 0, s, g.cstart, g.nx, nrows,
                       max_w < 1 ? 1 : max_w, (uint32_t)g.tile_max, t, (uint32_t)bound, overflow);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        if (ar == nullptr) dfree(t, s);
        return hip_status(e, "tiles launch");
    }
    *tiles = t;
    *cap = (uint32_t)bound;
    return CUTE_OK;
}

}  // namespace cute
