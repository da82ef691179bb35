// Host side of the C ABI: error reporting, the single pair count, and the
// estimators. Launch planning (thresholds, bands, LDS) is in plan.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdlib>
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

// The library's pool per device: freed blocks up to kPoolKeep bytes stay
// reserved for the next call; beyond that they go back to the device at the
// next synchronisation (large grids do not stay reserved after they are freed).
constexpr uint64_t kPoolKeep = 256ull << 20;
static hipMemPool_t g_pool[64] = {};

cute_status ensure_device_ready(int* device) {
    static std::mutex mu;
    static bool ready[64] = {false};
    int dev = 0;
    CUTE_HIP(hipGetDevice(&dev));
    *device = dev;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && !ready[dev]) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
            uint64_t thr = kPoolKeep;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            g_pool[dev] = pool;
        }
        ready[dev] = true;
    }
    return CUTE_OK;
}

bool inject_alloc_failure() {
    static std::atomic<uint64_t> calls{0};
    const char* v = std::getenv("CUTE_TEST_FAIL_ALLOC");
    if (v == nullptr) return false;
    const long n = std::strtol(v, nullptr, 10);
    if (n <= 0) return false;
    return (calls.fetch_add(1) + 1) % (uint64_t)n == 0;
}

cute_status dev_malloc_async(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (inject_alloc_failure())
        return fail(CUTE_E_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) +
                                              " bytes refused (CUTE_TEST_FAIL_ALLOC)");
    int dev = 0;
    CUTE_HIP(hipGetDevice(&dev));
    hipMemPool_t pool = (dev >= 0 && dev < 64) ? g_pool[dev] : nullptr;
    hipError_t e = pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_status(e, "device allocation");
    }
    return CUTE_OK;
}

cute_status DevArena::scratch_full(size_t need) const {
    return fail(CUTE_E_INVALID_ARG, "scratch area full: " + std::to_string(need) + " more bytes needed, " +
                                        std::to_string(cap_ - used_) + " of " + std::to_string(cap_) +
                                        " left");
}

struct StageBuf {
    unsigned char* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // recorded when the last lease ended
    int dev = -1;               // device of the event
};

static std::mutex g_stage_mu;
static std::vector<StageBuf*> g_stage_free;

cute_status HostStage::get(size_t bytes, unsigned char** p) {
    *p = nullptr;
    if (!b_) {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (!g_stage_free.empty()) {
            b_ = g_stage_free.back();
            g_stage_free.pop_back();
        }
    }
    if (!b_) {
        b_ = new (std::nothrow) StageBuf;
        if (!b_) return fail(CUTE_E_OUT_OF_MEMORY, "host allocation");
    }
    if (b_->done) CUTE_HIP(hipEventSynchronize(b_->done));
    if (bytes > b_->cap) {
        if (b_->p) (void)hipHostFree(b_->p);
        b_->p = nullptr;
        b_->cap = 0;
        const size_t cap = std::max<size_t>(bytes, 64 * 1024);
        CUTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&b_->p), cap, hipHostMallocDefault));
        b_->cap = cap;
    }
    *p = b_->p;
    return CUTE_OK;
}

HostStage::~HostStage() {
    if (!b_) return;
    int dev = -1;
    bool ok = hipGetDevice(&dev) == hipSuccess;
    if (ok && b_->dev != dev) {
        if (b_->done) (void)hipEventDestroy(b_->done);
        b_->done = nullptr;
        b_->dev = dev;
        if (hipEventCreateWithFlags(&b_->done, hipEventDisableTiming) != hipSuccess)
            b_->done = nullptr;
    }
    if (!ok || !b_->done || hipEventRecord(b_->done, s_) != hipSuccess) {
        // no event to wait on later: wait for the copies now
        (void)hipStreamSynchronize(s_);
        if (b_->done) {
            (void)hipEventDestroy(b_->done);
            b_->done = nullptr;
            b_->dev = -1;
        }
    }
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage_free.push_back(b_);
}

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

namespace {

// A radial count: redshifts per point (input order of each grid), the
// redshift-difference edges; the angular aperture is the reach of the THETA
// binning passed beside it.
struct RadialSpec {
    const double* ra;
    const double* rb;
    int on_device;
    int n;
    const double* edges;
    double aperture;
};

// One pair count; with max_tiles > 0 only an evenly spread sample of about
// max_tiles home tiles is counted (the tuner's sample).
// With fixed set, every device temporary is a slice of the caller's fixed
// area (nothing is allocated or freed, no pinned staging, no new events),
// the tiles are always built without a host wait, and a count whose
// temporaries would not fit is rejected before any work is enqueued.
cute_status count_impl(const cute_grid* ga, const cute_grid* gb, const cute_binning* bins,
                       cute_precision prec, uint64_t* counts, int32_t counts_on_device,
                       cute_count_stats* st, void* stream, uint32_t max_tiles,
                       double* sampled_share = nullptr, const RadialSpec* rad = nullptr,
                       const FixedArea* fixed = nullptr) {
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
    {
        // work on this stream follows the builds of both grids
        cute_status w;
        if ((w = grid_wait(ga, (hipStream_t)stream)) != CUTE_OK) return w;
        if (gb != ga && (w = grid_wait(gb, (hipStream_t)stream)) != CUTE_OK) return w;
    }
    const bool weighted = A.wt != nullptr || B.wt != nullptr;
    if (weighted && (A.wt == nullptr || B.wt == nullptr))
        return fail(CUTE_E_INVALID_ARG, "a pixel map pairs only with another pixel map");
    if (weighted && bins->kind != CUTE_BIN_THETA)
        return fail(CUTE_E_UNSUPPORTED, "pixel maps take a THETA binning");

    Plan pl;
    plan_binning(bins, pl);
    ItemGeom geo;
    if ((s = plan_item(A, B, is_auto, bins, pl, &geo)) != CUTE_OK) return s;
    plan_bands(bins, geo.em, pl);
    if (rad) {
        // the aperture binning gave the geometry; the histogram is over the
        // redshift difference, compared with the unsquared edges
        CountArgs& r = pl.a;
        const double c = 2.0 * std::sin(0.5 * rad->aperture);
        r.ap2 = c * c;
        r.top64 = r.ap2;
        pl.mode = M_RADIAL;
        pl.est = E_LIN;
        pl.T1.assign(rad->edges, rad->edges + rad->n + 1);
        pl.T2.assign(1, 0.0);
        pl.band1.assign(rad->n, make_float2(0.f, 0.f));
        pl.band2.assign(1, make_float2(0.f, 0.f));
        r.n1 = rad->n;
        r.n2 = 0;
        r.nbins = rad->n;
        r.n2p1 = 1;
    }
    if ((s = plan_lds(pl, 0)) != CUTE_OK) return s;
    CountArgs a = pl.a;
    apply_item(geo, &a);
    const int nbins = a.nbins;

    int dev = 0;
    if ((s = ensure_device_ready(&dev)) != CUTE_OK) return s;
    hipStream_t hs = (hipStream_t)stream;

    // ---- device buffers: one block, filled by one copy ------------------------
    // [T1 | T2 | B1 | B2 | stencil | args | counts, stats[4], head, tile count,
    //  tile-slot overflow]
    auto up16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    const size_t oT1 = 0;
    const size_t oT2 = oT1 + up16(pl.T1.size() * 8);
    const size_t oB1 = oT2 + up16(pl.T2.size() * 8);
    const size_t oB2 = oB1 + up16(pl.band1.size() * 8);
    const size_t oST = oB2 + up16(pl.band2.size() * 8);
    const size_t oAR = oST + up16(geo.stencil.size() * sizeof(int4));
    const size_t oWK = oAR + up16(sizeof(CountArgs));
    const size_t total = oWK + ((size_t)nbins + 7) * 8;
    if (fixed != nullptr) {
        if (rad != nullptr || max_tiles > 0)
            return fail(CUTE_E_INTERNAL, "fixed scratch serves plain counts only");
        // every temporary of the count, with the slot bound of its tiles
        const uint64_t bound = A.n > 0 && B.n > 0 ? tile_count_bound(A, geo.max_w) : 0;
        const size_t need = DevArena::cost<unsigned char>(total) +
                            2 * DevArena::cost<Tile>((size_t)bound) +
                            2 * DevArena::cost<uint32_t>((size_t)bound) +
                            DevArena::cost<uint32_t>(256);
        if (need > fixed->cap)
            return fail(CUTE_E_INVALID_ARG,
                        "this count needs " + std::to_string(need) + " bytes of scratch, more than "
                        "the " + std::to_string(fixed->cap) + " the no-allocation entry point holds");
    }
    DevArena mem_fixed(hs, fixed ? fixed->base : nullptr, fixed ? fixed->cap : 0);
    DevArena mem_pool(hs);
    DevArena& tmp = fixed ? mem_fixed : mem_pool;
    unsigned char* blob = nullptr;
    if ((s = tmp.get(&blob, total)) != CUTE_OK) return s;
    // pinned staging: [blob image | argument block | read-back of counts and
    // statistics]; the lease outlives every copy below (declared after tmp,
    // released first, which records its event after the copies)
    const size_t hArgs = up16(total), hBack = hArgs + up16(sizeof(CountArgs));
    HostStage stage(hs);
    std::vector<unsigned char> pageable;
    unsigned char* hb = nullptr;
    const size_t hbytes = hBack + ((size_t)nbins + 7) * 8;
    if (fixed) {
        // pageable host memory: no pinned allocation (the copies then wait)
        pageable.resize(hbytes);
        hb = pageable.data();
    } else if ((s = stage.get(hbytes, &hb)) != CUTE_OK) {
        return s;
    }
    // tables and zeroed counts in one copy (the argument block follows later)
    memset(hb, 0, total);
    memcpy(hb + oT1, pl.T1.data(), pl.T1.size() * 8);
    memcpy(hb + oT2, pl.T2.data(), pl.T2.size() * 8);
    memcpy(hb + oB1, pl.band1.data(), pl.band1.size() * 8);
    memcpy(hb + oB2, pl.band2.data(), pl.band2.size() * 8);
    if (!geo.stencil.empty())
        memcpy(hb + oST, geo.stencil.data(), geo.stencil.size() * sizeof(int4));
    CUTE_HIP(hipMemcpyAsync(blob, hb, total, hipMemcpyHostToDevice, hs));
    unsigned long long* work = reinterpret_cast<unsigned long long*>(blob + oWK);
    // the tile count and the slot-overflow flag, when the tiles are built
    // without a wait
    uint32_t* ntiles_dev = reinterpret_cast<uint32_t*>(work + nbins + 5);
    uint32_t* slot_overflow = reinterpret_cast<uint32_t*>(work + nbins + 6);
    CountArgs* dargs = reinterpret_cast<CountArgs*>(blob + oAR);
    if (rad) {
        // redshifts in each grid's sorted order
        double *rsa = nullptr, *rsb = nullptr;
        if ((s = tmp.get(&rsa, (size_t)A.n)) != CUTE_OK) return s;
        if ((s = gather_values(A, rad->ra, rad->on_device != 0, rsa, hs)) != CUTE_OK) return s;
        if (is_auto) {
            rsb = rsa;
        } else {
            if ((s = tmp.get(&rsb, (size_t)B.n)) != CUTE_OK) return s;
            if ((s = gather_values(B, rad->rb, rad->on_device != 0, rsb, hs)) != CUTE_OK) return s;
        }
        a.rA = rsa;
        a.rB = rsb;
    }
    const int4* dst = geo.stencil.empty() ? nullptr : reinterpret_cast<const int4*>(blob + oST);
    a.stencil = dst;
    a.nst = (int)geo.stencil.size();
    a.T1 = reinterpret_cast<const double*>(blob + oT1);
    a.T2 = reinterpret_cast<const double*>(blob + oT2);
    a.band1 = reinterpret_cast<const float2*>(blob + oB1);
    a.band2 = reinterpret_cast<const float2*>(blob + oB2);
    a.counts = work;
    a.stats = work + nbins;
    a.work_head = reinterpret_cast<uint32_t*>(work + nbins + 4);

    Tile* tiles = nullptr;
    uint32_t ntiles = 0;   // the count, or with dev_count the capacity of tiles
    bool dev_count = false;
    // tiles from the fixed area are never freed
    auto drop_tiles = [&]() {
        if (!fixed) dfree(tiles, hs);
        tiles = nullptr;
    };
    if (fixed && A.n > 0 && B.n > 0) {
        // slots without a host wait, compacted on the device (longest first
        // when the neighbour rows are tabulated)
        if ((s = build_tiles_nowait(A, geo.max_w, hs, &tiles, &ntiles, slot_overflow, &tmp)) !=
            CUTE_OK)
            return s;
        dev_count = true;
    } else if (A.n > 0 && B.n > 0) {
        GridHost At = A;
        // Too few tiles to give every wave slot of the chip two: cut them
        // shorter (default tile size only; not below 16 points, where the
        // per-tile neighbour walk starts to dominate).
        int ncu = 0;
        const bool may_shrink =
            A.tile_auto && max_tiles == 0 &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess;
        const uint64_t want = (uint64_t)ncu * 16u * 2u;
        // Every tile holds at most tile_max points. When that many tiles
        // already fill the chip and the host-side bound on their number is
        // modest, build them into slots without waiting for their count; the
        // longest-first reordering compacts them and leaves the count on the
        // device.
        const uint64_t min_tiles = ((uint64_t)A.n + At.tile_max - 1) / At.tile_max;
        const uint64_t bound = tile_count_bound(At, geo.max_w);
        if (max_tiles == 0 && dst != nullptr && a.nst > 0 && (!may_shrink || min_tiles >= want) &&
            bound <= std::max<uint64_t>(65536, 4 * min_tiles)) {
            if ((s = build_tiles_nowait(At, geo.max_w, hs, &tiles, &ntiles, slot_overflow)) !=
                CUTE_OK)
                return s;
            dev_count = true;
        } else {
            if ((s = build_tiles(At, geo.max_w, hs, &tiles, &ntiles)) != CUTE_OK) return s;
            while (may_shrink && ntiles < want && At.tile_max > 16) {
                At.tile_max = std::max(16, At.tile_max / 2);
                drop_tiles();
                if ((s = build_tiles(At, geo.max_w, hs, &tiles, &ntiles)) != CUTE_OK) return s;
            }
        }
    }
    if ((s = order_tiles(A, B, dst, a.nst, is_auto, geo.periodic != 0, &tiles, ntiles, hs,
                         dev_count ? ntiles_dev : nullptr, fixed ? &tmp : nullptr)) != CUTE_OK) {
        drop_tiles();
        return s;
    }
    const uint32_t tile_stride = max_tiles > 0 ? (ntiles + max_tiles - 1) / max_tiles : 1;
    if (tile_stride > 1 && ntiles > 0) {
        // keep every tile_stride-th tile (in place: a stream-ordered round trip)
        std::vector<Tile> h(ntiles);
        hipError_t e = hipMemcpyAsync(h.data(), tiles, ntiles * sizeof(Tile), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) {
            drop_tiles();
            return hip_status(e, "tile sample");
        }
        uint32_t k = 0;
        for (uint32_t t = 0; t < ntiles; t += tile_stride) h[k++] = h[t];
        if (sampled_share) *sampled_share = (double)k / (double)ntiles;
        ntiles = k;
        e = hipMemcpyAsync(tiles, h.data(), ntiles * sizeof(Tile), hipMemcpyHostToDevice, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) {
            drop_tiles();
            return hip_status(e, "tile sample");
        }
    }
    a.tiles = tiles;
    a.ntiles = ntiles;
    a.ntiles_dev = dev_count ? ntiles_dev : nullptr;
    a.self = dargs;
    a.wA = A.wt;
    a.wB = B.wt;
    memcpy(hb + hArgs, &a, sizeof(a));
    CUTE_HIP(hipMemcpyAsync(dargs, hb + hArgs, sizeof(a), hipMemcpyHostToDevice, hs));

    // launch, then the copies, then one wait (the end event is read after it)
    int grid = 0;
    EventTimer timer(hs, fixed ? fixed->events : nullptr);
    if (ntiles > 0) {
        s = launch_count(a, pl.mode, (int)prec, pl.est, kWgWaves, pl.lds, hs, &grid);
        if (s != CUTE_OK) {
            drop_tiles();
            return s;
        }
    }
    // objects that share a pixel: zero separation, in the first bin if it
    // starts at zero
    if (weighted && is_auto && bins->edges1[0] == 0.0 && sampled_share == nullptr) {
        if ((s = add_pixel_self_pairs(A, work, hs)) != CUTE_OK) {
            drop_tiles();
            return s;
        }
    }
    timer.stop();
    drop_tiles();
    if (counts_on_device)
        CUTE_HIP(hipMemcpyAsync(counts, work, (size_t)nbins * 8, hipMemcpyDeviceToDevice, hs));
    // one read-back of [counts | statistics, head, tile count] (the counts
    // only when they go to the host or their sum is asked for)
    const bool back_counts = !counts_on_device || st;
    const unsigned long long* hw = reinterpret_cast<const unsigned long long*>(hb + hBack);
    const unsigned long long* hst = hw + (back_counts ? nbins : 0);
    CUTE_HIP(hipMemcpyAsync(hb + hBack, back_counts ? work : work + nbins,
                            ((back_counts ? (size_t)nbins : 0) + 7) * 8, hipMemcpyDeviceToHost, hs));
    CUTE_HIP(hipStreamSynchronize(hs));
    const double ms = ntiles > 0 ? timer.elapsed_ms() : 0.0;
    if (!counts_on_device) memcpy(counts, hw, (size_t)nbins * 8);
    if (st) {
        st->pair_evals = hst[0];
        st->retests = hst[1];
        st->flips = hst[2];
        st->tiles = hst[3];
        st->ms_count = ms;
        uint64_t tot = 0;
        for (int k = 0; k < nbins; k++) tot += (uint64_t)hw[k];
        st->pairs_in_range = tot;
    }
    if (dev_count && hst[6] != 0) return fail(CUTE_E_INTERNAL, "tile slots overflowed");
    const uint64_t want_tiles = dev_count ? (uint64_t)hst[5] : (uint64_t)ntiles;
    if (hst[3] != want_tiles) return fail(CUTE_E_INTERNAL, "not every tile was processed");
    return CUTE_OK;
}

}  // namespace

cute_status cute::count_pairs_fixed(const cute_grid* a, const cute_grid* b,
                                    const cute_binning* bins, cute_precision prec,
                                    uint64_t* counts, int32_t counts_on_device,
                                    cute_count_stats* st, void* stream, const FixedArea* fixed) {
    if (!fixed || !fixed->base) return fail(CUTE_E_INTERNAL, "no fixed scratch area");
    return count_impl(a, b, bins, prec, counts, counts_on_device, st, stream, 0, nullptr, nullptr,
                      fixed);
}

extern "C" cute_status cute_count_pairs(const cute_grid* ga, const cute_grid* gb,
                                        const cute_binning* bins, cute_precision prec,
                                        uint64_t* counts, int32_t counts_on_device,
                                        cute_count_stats* st, void* stream) {
    return count_impl(ga, gb, bins, prec, counts, counts_on_device, st, stream, 0);
}

extern "C" cute_status cute_count_radial(const cute_grid* a, const double* ra, const cute_grid* b,
                                         const double* rb, int32_t r_on_device, double aperture,
                                         int32_t n_bins, const double* edges, uint64_t* counts,
                                         int32_t counts_on_device, cute_count_stats* st,
                                         void* stream) {
    if (!a) return fail(CUTE_E_INVALID_ARG, "grid a is NULL");
    const bool is_auto = (b == nullptr || b == a);
    if ((a->h.n > 0 && !ra) || (!is_auto && b->h.n > 0 && !rb))
        return fail(CUTE_E_INVALID_ARG, "redshift pointer is NULL");
    if (!(aperture > 0.0 && aperture <= 3.14159265358979323846))
        return fail(CUTE_E_INVALID_ARG, "aperture must be in (0, pi]");
    if (n_bins < 1 || n_bins > (1 << 20) || !edges)
        return fail(CUTE_E_INVALID_ARG, "need n_bins >= 1 and n_bins + 1 edges");
    for (int k = 0; k <= n_bins; k++)
        if (!std::isfinite(edges[k]) || edges[k] < 0.0 || (k > 0 && !(edges[k - 1] < edges[k])))
            return fail(CUTE_E_INVALID_ARG, "edges must be finite, >= 0 and strictly increasing");
    if (a->h.wt != nullptr || (!is_auto && b->h.wt != nullptr))
        return fail(CUTE_E_UNSUPPORTED, "radial counts take catalogs, not pixel maps");
    const double ae[2] = {0.0, aperture};
    cute_binning ab;
    memset(&ab, 0, sizeof(ab));
    ab.kind = CUTE_BIN_THETA;
    ab.n1 = 1;
    ab.edges1 = ae;
    RadialSpec rs{ra, is_auto ? ra : rb, r_on_device, n_bins, edges, aperture};
    return count_impl(a, b, &ab, CUTE_PREC_FP64, counts, counts_on_device, st, stream, 0, nullptr,
                      &rs);
}

extern "C" cute_status cute_tune_grid(const double* x, const double* y, const double* z,
                                      int64_t n, const cute_grid_params* p,
                                      const cute_binning* bins, cute_precision prec,
                                      int32_t n_cell, const double* cells, int32_t n_tile,
                                      const int32_t* tiles, void* stream, double* best_cell,
                                      int32_t* best_tile, double* ms) {
    if (!best_cell || !best_tile) return fail(CUTE_E_INVALID_ARG, "best_cell or best_tile is NULL");
    if (!p) return fail(CUTE_E_INVALID_ARG, "params is NULL");
    cute_status s = validate_binning(bins);
    if (s != CUTE_OK) return s;
    if (n_cell < 0 || n_cell > 64 || (n_cell > 0 && !cells) || n_tile < 0 || n_tile > 64 ||
        (n_tile > 0 && !tiles))
        return fail(CUTE_E_INVALID_ARG, "n_cell and n_tile must be in [0, 64] with arrays given");
    Plan pl;
    plan_binning(bins, pl);
    const double rmax = bins->kind == CUTE_BIN_THETA ? bins->edges1[bins->n1] : pl.rmax;
    std::vector<double> cand;
    if (n_cell > 0) {
        for (int i = 0; i < n_cell; i++) {
            if (!(cells[i] >= 0.0) || !std::isfinite(cells[i]))
                return fail(CUTE_E_INVALID_ARG, "cell sides must be finite and >= 0");
            cand.push_back(cells[i]);
        }
    } else {
        cand.push_back(0.0);  // the library's density rule
        for (double f : {1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6}) cand.push_back(rmax * f);
    }
    std::vector<int> tsz;
    if (n_tile > 0) {
        for (int i = 0; i < n_tile; i++) {
            if (tiles[i] < 1 || tiles[i] > 64)
                return fail(CUTE_E_INVALID_ARG, "tile sizes must be in 1..64");
            tsz.push_back(tiles[i]);
        }
    } else {
        tsz = {32, 64};
    }
    // a sample of home tiles (longest-first order, evenly spread), large
    // enough that the persistent waves take several each: the time then
    // tracks throughput, not the longest single tile
    const uint32_t sample = 32768;
    std::vector<uint64_t> counts((size_t)pl.a.nbins);
    std::vector<double> tms(cand.size() * tsz.size(), INFINITY);
    double best_ms = INFINITY;
    for (size_t i = 0; i < cand.size() * tsz.size(); i++) {
        cute_grid_params q = *p;
        q.cell_size = cand[i / tsz.size()];
        q.tile_points = tsz[i % tsz.size()];
        if (q.r_max < rmax) q.r_max = rmax;
        cute_grid* g = nullptr;
        s = cute_build_grid(x, y, z, n, &q, stream, &g);
        double t = INFINITY;
        if (s == CUTE_OK) {
            for (int rep = 0; rep < 2 && s == CUTE_OK; rep++) {
                cute_count_stats st;
                double share = 1.0;  // the time is scaled to the whole count
                s = count_impl(g, nullptr, bins, prec, counts.data(), 0, &st, stream, sample,
                               &share);
                if (s == CUTE_OK) t = std::min(t, st.ms_count / share);
            }
            cute_free_grid(g);
        }
        if (s == CUTE_E_OUT_OF_MEMORY || s == CUTE_E_DEVICE) return s;
        if (ms) ms[i] = s == CUTE_OK ? t : NAN;  // a rejected pair is NaN
        if (s == CUTE_OK) {
            tms[i] = t;
            best_ms = std::min(best_ms, t);
        }
    }
    if (!std::isfinite(best_ms)) return fail(CUTE_E_INVALID_ARG, "no candidate is usable");
    // timings differ by a percent or two from run to run: among the pairs
    // within 2 % of the fastest, take the largest tile, then the first cell
    // side in the candidate order, so that the choice is stable
    int best_i = -1;
    std::vector<size_t> tord(tsz.size());
    for (size_t k = 0; k < tsz.size(); k++) tord[k] = k;
    std::stable_sort(tord.begin(), tord.end(), [&](size_t u, size_t v) { return tsz[u] > tsz[v]; });
    for (size_t k = 0; k < tord.size() && best_i < 0; k++)
        for (size_t c = 0; c < cand.size() && best_i < 0; c++) {
            const size_t i = c * tsz.size() + tord[k];
            if (tms[i] <= best_ms * 1.02) best_i = (int)i;
        }
    *best_cell = cand[best_i / tsz.size()];
    *best_tile = tsz[best_i % tsz.size()];
    return CUTE_OK;
}

// ---------------------------------------------------------------------------
// Estimators (Sec. 2.2) and multipoles (Sec. 2.1), host only.
// ---------------------------------------------------------------------------
// __int128 -> double through the compiler's correctly rounded conversion
static double i128_to_double(__int128 v) { return static_cast<double>(v); }

extern "C" cute_status cute_fp32_decision_tables(const cute_binning* bins, const double* err,
                                                 float* band1, float* band2, float* consts) {
    cute_status s;
    if ((s = validate_binning(bins)) != CUTE_OK) return s;
    const bool mid = bins->kind == CUTE_BIN_SIGMAPI ||
                     (bins->kind == CUTE_BIN_RMU && bins->los == CUTE_LOS_MIDPOINT);
    if (!mid) return fail(CUTE_E_UNSUPPORTED, "decision tables are reported for the midpoint line of sight only");
    if (!err || !band1 || !band2 || !consts) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    for (int k = 0; k < 4; k++)
        if (!std::isfinite(err[k]) || err[k] < 0.0)
            return fail(CUTE_E_INVALID_ARG, "error bounds must be finite and >= 0");
    Plan pl;
    plan_binning(bins, pl);
    ErrModel em;
    em.ec = err[0];
    em.ec64 = err[1];
    em.el = err[2];
    em.el64 = err[3];
    plan_bands(bins, em, pl);
    for (int k = 0; k < bins->n1; k++) {
        band1[2 * k] = pl.band1[k].x;
        band1[2 * k + 1] = pl.band1[k].y;
    }
    for (int k = 0; k < bins->n2; k++) {
        band2[2 * k] = pl.band2[k].x;
        band2[2 * k + 1] = pl.band2[k].y;
    }
    const CountArgs& a = pl.a;
    const float c[kDecisionConsts] = {a.skip32, a.llg, a.spK1, a.spK0, a.sp_wstop, a.sp_wptop,
                                      a.sp_wsbot, a.sp_wpbot, (float)a.sp_low, a.dA0, a.dA1, a.dA2,
                                      a.dB0, a.dB1, a.dB2, a.dC2, a.dC0};
    for (int k = 0; k < kDecisionConsts; k++) consts[k] = c[k];
    return CUTE_OK;
}

extern "C" cute_status cute_fp32_zlos_constants(const cute_binning* bins, const double* err,
                                                float* consts) {
    cute_status s;
    if ((s = validate_binning(bins)) != CUTE_OK) return s;
    if (bins->kind != CUTE_BIN_RMU || bins->los != CUTE_LOS_Z)
        return fail(CUTE_E_UNSUPPORTED, "z line-of-sight constants are reported for RMU with CUTE_LOS_Z only");
    if (!err || !consts) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    for (int k = 0; k < 2; k++)
        if (!std::isfinite(err[k]) || err[k] < 0.0)
            return fail(CUTE_E_INVALID_ARG, "error bounds must be finite and >= 0");
    Plan pl;
    plan_binning(bins, pl);
    ErrModel em;
    em.ec = err[0];
    em.ec64 = err[1];
    plan_bands(bins, em, pl);
    const CountArgs& a = pl.a;
    const float c[9] = {a.e1a, a.s1, a.e2a, a.s2, a.rB0, a.muB1, a.muB0, a.out_hi, (float)pl.est};
    for (int k = 0; k < 9; k++) consts[k] = c[k];
    return CUTE_OK;
}

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
    // With nd, nr < 2^31 (the size limit of a grid) and every count at most
    // the number of pairs it can hold (DD <= nd(nd-1)/2, DR <= nd nr,
    // RR <= nr(nr-1)/2), each product below is under 2^124 and the
    // numerator N_r(N_r-1)DD - (N_r-1)(N_d-1)DR + N_d(N_d-1)RR lies in
    // (-2^124, 2^124): no 128-bit overflow.
    if (nd >= ((int64_t)1 << 31) || nr >= ((int64_t)1 << 31))
        return fail(CUTE_E_INVALID_ARG, "catalog sizes must be below 2^31");
    const uint64_t max_dd = (uint64_t)nd * (uint64_t)(nd - 1) / 2u;
    const uint64_t max_rr = (uint64_t)nr * (uint64_t)(nr - 1) / 2u;
    const uint64_t max_dr = (uint64_t)nd * (uint64_t)nr;
    const __int128 cdd = (__int128)nr * (nr - 1);   // multiplies DD
    const __int128 cdr = (__int128)(nr - 1) * (nd - 1);
    const __int128 crr = (__int128)nd * (nd - 1);   // multiplies RR (and the denominator)
    for (int k = 0; k < nbins; k++) {
        if (rr[k] == 0) {
            xi[k] = NAN;
            continue;
        }
        if (dd[k] > max_dd || rr[k] > max_rr || (dr && dr[k] > max_dr))
            return fail(CUTE_E_INVALID_ARG,
                        "a count exceeds the number of pairs of its catalogs (DD <= nd(nd-1)/2, "
                        "DR <= nd nr, RR <= nr(nr-1)/2)");
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
