// Host side of the batched counts: planning of the items, launch groups (one
// per distinct binning), work chunks ordered by estimated cost, sorted-order
// mask bits, the device counts, and the HIP graph that replays the launches.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "cute_internal.h"
#include "runtime.h"

using namespace cute;

namespace {

// Items of one binning, counted by one persistent launch.
struct Group {
    Plan pl;
    int grid = 0;                    // workgroups
    BatchArgs ba;                    // device pointers filled at creation
    std::vector<int> items;          // item indices, largest estimated cost first
    double *dT1 = nullptr, *dT2 = nullptr;
    float2 *dB1 = nullptr, *dB2 = nullptr;
    uint32_t* dchunks = nullptr;
};

}  // namespace

struct cute_batch {
    int device = 0;
    int prec = 0;
    int n_items = 0;
    std::vector<Group> groups;
    std::vector<int64_t> words;      // count words per item
    std::vector<int64_t> offset;     // offset of each item's counts
    std::vector<uint32_t> ntiles;    // home tiles per item
    int64_t total_words = 0;
    unsigned long long* work = nullptr;   // counts | stats (4 per item) | chunk heads
    size_t work_words = 0;
    CountArgs* dargs = nullptr;      // one per item
    std::vector<void*> owned;        // device allocations (hipMalloc)
    std::vector<Tile*> tiles;        // per item (stream-ordered allocations)
    hipStream_t cap = nullptr;       // private stream used for capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <typename T>
cute_status owned_alloc(cute_batch* b, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (inject_alloc_failure())
        return fail(CUTE_E_OUT_OF_MEMORY, "device allocation refused (CUTE_TEST_FAIL_ALLOC)");
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) return hip_status(e, "hipMalloc");
    b->owned.push_back(*p);
    return CUTE_OK;
}

void release(cute_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (Tile* t : b->tiles)
        if (t) (void)hipFreeAsync(t, nullptr);  // stream-ordered allocations
    (void)hipStreamSynchronize(nullptr);
    for (void* p : b->owned) (void)hipFree(p);
    delete b;
}

// Enqueue one run: clear counts, statistics and chunk heads, then one
// persistent launch per group. No allocation, memset or synchronisation.
cute_status enqueue_run(cute_batch* b, hipStream_t s) {
    cute_status st = zero_u64(b->work, b->work_words, s);
    if (st != CUTE_OK) return st;
    for (const Group& g : b->groups) {
        if (g.ba.nchunks == 0) continue;
        st = batch_launch(g.ba, g.pl.mode, b->prec, g.pl.est, g.grid, g.pl.lds, s);
        if (st != CUTE_OK) return st;
    }
    return CUTE_OK;
}

cute_status create(const cute_batch_item* items, int32_t n_items, cute_precision prec,
                   hipStream_t hs, cute_batch* b) {
    cute_status s;
    if (prec != CUTE_PREC_FP64 && prec != CUTE_PREC_FP32_EDGE && prec != CUTE_PREC_FP32_ONLY)
        return fail(CUTE_E_INVALID_ARG, "unknown precision");
    b->prec = (int)prec;
    b->n_items = n_items;
    std::vector<ItemGeom> geo(n_items);
    std::vector<int> gid(n_items, -1);
    // ---- validate and group the items by binning ---------------------------
    for (int i = 0; i < n_items; i++) {
        const cute_batch_item& it = items[i];
        if (!it.a) return fail(CUTE_E_INVALID_ARG, "item " + std::to_string(i) + ": grid a is NULL");
        if ((s = validate_binning(it.bins)) != CUTE_OK) return s;
        const bool is_auto = it.b == nullptr || it.b == it.a;
        const cute_grid* gb = is_auto ? it.a : it.b;
        if (it.a->h.wt != nullptr || gb->h.wt != nullptr)
            return fail(CUTE_E_UNSUPPORTED, "item " + std::to_string(i) + ": pixel maps are counted one at a time");
        int g = -1;
        for (size_t k = 0; k < b->groups.size(); k++) {
            const int first = b->groups[k].items[0];
            if (same_binning(items[first].bins, it.bins)) {
                g = (int)k;
                break;
            }
        }
        if (g < 0) {
            b->groups.emplace_back();
            g = (int)b->groups.size() - 1;
            plan_binning(it.bins, b->groups[g].pl);
        }
        Group& G = b->groups[g];
        if ((s = plan_item(it.a->h, gb->h, is_auto, it.bins, G.pl, &geo[i])) != CUTE_OK) {
            set_error("item " + std::to_string(i) + ": " + std::string(cute_last_error()));
            return s;
        }
        G.items.push_back(i);
        gid[i] = g;
        const int64_t w = (int64_t)G.pl.a.nbins;
        b->words.push_back(w);
        b->offset.push_back(b->total_words);
        b->total_words += w;
    }
    // ---- bands (one error model per group), LDS plan, kernel attributes -----
    int dev = 0, ncu = 0;
    if ((s = ensure_device_ready(&dev)) != CUTE_OK) return s;
    // the set-up work on hs (and every replay, which follows it) comes after
    // the builds of the grids
    for (int i = 0; i < n_items; i++) {
        if ((s = grid_wait(items[i].a, hs)) != CUTE_OK) return s;
        if (items[i].b && items[i].b != items[i].a && (s = grid_wait(items[i].b, hs)) != CUTE_OK)
            return s;
    }
    b->device = dev;
    CUTE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    for (Group& G : b->groups) {
        ErrModel em = geo[G.items[0]].em;
        for (int i : G.items) em = max_err(em, geo[i].em);
        plan_bands(items[G.items[0]].bins, em, G.pl);
        if ((s = plan_lds(G.pl, 16)) != CUTE_OK) return s;
        int per_cu = 1;
        if ((s = batch_prepare(G.pl.mode, b->prec, G.pl.est, G.pl.lds, &per_cu)) != CUTE_OK) return s;
        G.grid = per_cu * ncu;
        std::stable_sort(G.items.begin(), G.items.end(),
                         [&](int x, int y) { return geo[x].cost > geo[y].cost; });
    }
    // ---- device memory -------------------------------------------------------
    b->work_words = (size_t)b->total_words + 4 * (size_t)n_items + b->groups.size();
    if ((s = owned_alloc(b, &b->work, b->work_words)) != CUTE_OK) return s;
    if ((s = owned_alloc(b, &b->dargs, (size_t)n_items)) != CUTE_OK) return s;
    for (Group& G : b->groups) {
        if ((s = owned_alloc(b, &G.dT1, G.pl.T1.size())) != CUTE_OK) return s;
        if ((s = owned_alloc(b, &G.dT2, G.pl.T2.size())) != CUTE_OK) return s;
        if ((s = owned_alloc(b, &G.dB1, G.pl.band1.size())) != CUTE_OK) return s;
        if ((s = owned_alloc(b, &G.dB2, G.pl.band2.size())) != CUTE_OK) return s;
        CUTE_HIP(hipMemcpyAsync(G.dT1, G.pl.T1.data(), G.pl.T1.size() * 8, hipMemcpyHostToDevice, hs));
        CUTE_HIP(hipMemcpyAsync(G.dT2, G.pl.T2.data(), G.pl.T2.size() * 8, hipMemcpyHostToDevice, hs));
        CUTE_HIP(hipMemcpyAsync(G.dB1, G.pl.band1.data(), G.pl.band1.size() * 8,
                                hipMemcpyHostToDevice, hs));
        CUTE_HIP(hipMemcpyAsync(G.dB2, G.pl.band2.data(), G.pl.band2.size() * 8,
                                hipMemcpyHostToDevice, hs));
    }
    // ---- per item: tiles, mask bits, arguments --------------------------------
    b->tiles.assign(n_items, nullptr);
    b->ntiles.assign(n_items, 0);
    std::vector<CountArgs> args(n_items);
    for (int i = 0; i < n_items; i++) {
        const cute_batch_item& it = items[i];
        const bool is_auto = it.b == nullptr || it.b == it.a;
        const GridHost& A = it.a->h;
        const GridHost& B = is_auto ? it.a->h : it.b->h;
        const Group& G = b->groups[gid[i]];
        CountArgs& a = args[i];
        a = G.pl.a;
        apply_item(geo[i], &a);
        a.T1 = G.dT1;
        a.T2 = G.dT2;
        a.band1 = G.dB1;
        a.band2 = G.dB2;
        a.self = b->dargs + i;
        a.counts = b->work + b->offset[i];
        a.stats = b->work + b->total_words + 4 * (size_t)i;
        if (A.n > 0 && B.n > 0) {
            Tile* t = nullptr;
            uint32_t nt = 0;
            if ((s = build_tiles(A, geo[i].max_w, hs, &t, &nt)) != CUTE_OK) return s;
            b->tiles[i] = t;
            b->ntiles[i] = nt;
        }
        a.stencil = nullptr;
        a.nst = (int)geo[i].stencil.size();
        if (a.nst > 0) {
            int4* dst = nullptr;
            if ((s = owned_alloc(b, &dst, geo[i].stencil.size())) != CUTE_OK) return s;
            CUTE_HIP(hipMemcpyAsync(dst, geo[i].stencil.data(), geo[i].stencil.size() * sizeof(int4),
                                    hipMemcpyHostToDevice, hs));
            a.stencil = dst;
            // heavy tiles first within the item
            if ((s = order_tiles(A, B, dst, a.nst, is_auto, geo[i].periodic != 0, &b->tiles[i],
                                 b->ntiles[i], hs)) != CUTE_OK)
                return s;
        }
        a.tiles = b->tiles[i];
        a.ntiles = b->ntiles[i];
        // masks -> sorted-order bits
        const uint8_t* masks[2] = {it.mask_a, is_auto ? nullptr : it.mask_b};
        const GridHost* gh[2] = {&A, &B};
        const uint32_t* bits[2] = {nullptr, nullptr};
        for (int side = 0; side < 2; side++) {
            if (!masks[side] || gh[side]->n == 0) continue;
            const size_t n = (size_t)gh[side]->n;
            uint32_t* mb = nullptr;
            if ((s = owned_alloc(b, &mb, (n + 31) / 32)) != CUTE_OK) return s;
            const uint8_t* src = masks[side];
            uint8_t* tmp = nullptr;
            if (!it.masks_on_device) {
                if ((s = dalloc(&tmp, n, hs)) != CUTE_OK) return s;
                const hipError_t e = hipMemcpyAsync(tmp, src, n, hipMemcpyHostToDevice, hs);
                if (e != hipSuccess) {
                    dfree(tmp, hs);
                    return hip_status(e, "mask copy");
                }
                src = tmp;
            }
            s = mask_bits(src, *gh[side], mb, hs);
            if (tmp) dfree(tmp, hs);
            if (s != CUTE_OK) return s;
            bits[side] = mb;
        }
        a.mbA = bits[0];
        a.mbB = is_auto ? bits[0] : bits[1];
    }
    CUTE_HIP(hipMemcpyAsync(b->dargs, args.data(), sizeof(CountArgs) * (size_t)n_items,
                            hipMemcpyHostToDevice, hs));
    // ---- chunks: runs of home tiles of one item, largest items first --------
    size_t head_slot = (size_t)b->total_words + 4 * (size_t)n_items;
    std::vector<std::vector<uint32_t>> chunk_lists(b->groups.size());  // alive until the sync
    for (size_t gi = 0; gi < b->groups.size(); gi++) {
        Group& G = b->groups[gi];
        uint64_t total = 0;
        for (int i : G.items) total += b->ntiles[i];
        // about 8 chunks per workgroup, 4 to 64 tiles each
        uint64_t per = total / ((uint64_t)std::max(G.grid, 1) * 8);
        per = std::max<uint64_t>(4, std::min<uint64_t>(64, per));
        std::vector<uint32_t>& ch = chunk_lists[gi];
        for (int i : G.items)
            for (uint64_t t0 = 0; t0 < b->ntiles[i]; t0 += per) {
                const uint64_t t1 = std::min<uint64_t>(t0 + per, b->ntiles[i]);
                ch.push_back((uint32_t)i);
                ch.push_back((uint32_t)t0);
                ch.push_back((uint32_t)t1);
                ch.push_back(0u);
            }
        const uint32_t nch = (uint32_t)(ch.size() / 4);
        if ((s = owned_alloc(b, &G.dchunks, std::max<size_t>(ch.size(), 4))) != CUTE_OK) return s;
        if (nch)
            CUTE_HIP(hipMemcpyAsync(G.dchunks, ch.data(), ch.size() * 4, hipMemcpyHostToDevice, hs));
        G.grid = (int)std::min<uint64_t>((uint64_t)G.grid, std::max<uint32_t>(nch, 1u));
        BatchArgs& ba = G.ba;
        memset(&ba, 0, sizeof(ba));
        ba.items = b->dargs;
        ba.chunks = G.dchunks;
        ba.nchunks = nch;
        ba.head = reinterpret_cast<uint32_t*>(b->work + head_slot++);
        ba.n1 = G.pl.a.n1;
        ba.n2 = G.pl.a.n2;
        ba.nbins = G.pl.a.nbins;
        ba.copies = G.pl.a.copies;
        ba.hist_words = G.pl.a.hist_words;
        ba.T1 = G.dT1;
        ba.T2 = G.dT2;
        ba.band1 = G.dB1;
        ba.band2 = G.dB2;
    }
    CUTE_HIP(hipStreamSynchronize(hs));
    // ---- capture one run in a graph ----------------------------------------------
    CUTE_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    CUTE_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    s = enqueue_run(b, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (s != CUTE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture");
    b->graph = g;
    CUTE_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return CUTE_OK;
}

}  // namespace

extern "C" cute_status cute_batch_create(const cute_batch_item* items, int32_t n_items,
                                         cute_precision prec, void* stream, cute_batch** out) {
    if (!out) return fail(CUTE_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!items || n_items < 1) return fail(CUTE_E_INVALID_ARG, "no items");
    cute_batch* b = new cute_batch();
    cute_status s = create(items, n_items, prec, (hipStream_t)stream, b);
    if (s != CUTE_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release(b);
        return s;
    }
    *out = b;
    return CUTE_OK;
}

extern "C" cute_status cute_batch_run(cute_batch* b, int32_t flags, void* stream) {
    if (!b) return fail(CUTE_E_INVALID_ARG, "batch is NULL");
    hipStream_t hs = (hipStream_t)stream;
    if (flags == CUTE_BATCH_EAGER) return enqueue_run(b, hs);
    if (flags != CUTE_BATCH_GRAPH) return fail(CUTE_E_INVALID_ARG, "unknown flags");
    CUTE_HIP(hipGraphLaunch(b->exec, hs));
    return CUTE_OK;
}

extern "C" cute_status cute_batch_layout(const cute_batch* b, int32_t item, int64_t* words,
                                         int64_t* offset) {
    if (!b) return fail(CUTE_E_INVALID_ARG, "batch is NULL");
    if (item < -1 || item >= b->n_items) return fail(CUTE_E_INVALID_ARG, "item out of range");
    if (words) *words = item < 0 ? b->total_words : b->words[item];
    if (offset) *offset = item < 0 ? 0 : b->offset[item];
    return CUTE_OK;
}

extern "C" cute_status cute_batch_counts(const cute_batch* b, int32_t item, uint64_t* out,
                                         int32_t on_device, void* stream) {
    if (!b || !out) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    if (item < -1 || item >= b->n_items) return fail(CUTE_E_INVALID_ARG, "item out of range");
    hipStream_t hs = (hipStream_t)stream;
    const int64_t w = item < 0 ? b->total_words : b->words[item];
    const int64_t o = item < 0 ? 0 : b->offset[item];
    CUTE_HIP(hipMemcpyAsync(out, b->work + o, (size_t)w * 8,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, hs));
    if (!on_device) CUTE_HIP(hipStreamSynchronize(hs));
    return CUTE_OK;
}

extern "C" cute_status cute_batch_stats(const cute_batch* b, int32_t item, cute_count_stats* st,
                                        void* stream) {
    if (!b || !st) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    if (item < -1 || item >= b->n_items) return fail(CUTE_E_INVALID_ARG, "item out of range");
    hipStream_t hs = (hipStream_t)stream;
    std::vector<unsigned long long> h(b->work_words);
    CUTE_HIP(hipMemcpyAsync(h.data(), b->work, b->work_words * 8, hipMemcpyDeviceToHost, hs));
    CUTE_HIP(hipStreamSynchronize(hs));
    memset(st, 0, sizeof(*st));
    bool complete = true;
    for (int i = 0; i < b->n_items; i++) {
        if (item >= 0 && i != item) continue;
        const unsigned long long* sv = h.data() + b->total_words + 4 * (size_t)i;
        st->pair_evals += sv[0];
        st->retests += sv[1];
        st->flips += sv[2];
        st->tiles += sv[3];
        for (int64_t k = 0; k < b->words[i]; k++) st->pairs_in_range += h[b->offset[i] + k];
        complete = complete && sv[3] == b->ntiles[i];
    }
    if (!complete) return fail(CUTE_E_INTERNAL, "not every tile was processed");
    return CUTE_OK;
}

extern "C" void cute_batch_free(cute_batch* b) { release(b); }

extern "C" cute_status cute_count_pairs_batched(const cute_batch_item* items, int32_t n_items,
                                                cute_precision prec, uint64_t* const* counts,
                                                int32_t counts_on_device, cute_count_stats* st,
                                                void* stream) {
    if (!counts) return fail(CUTE_E_INVALID_ARG, "counts is NULL");
    for (int i = 0; i < n_items; i++)
        if (!counts[i]) return fail(CUTE_E_INVALID_ARG, "counts[" + std::to_string(i) + "] is NULL");
    cute_batch* b = nullptr;
    cute_status s = cute_batch_create(items, n_items, prec, stream, &b);
    if (s != CUTE_OK) return s;
    hipStream_t hs = (hipStream_t)stream;
    double ms = 0.0;
    {
        EventTimer timer(hs);
        s = cute_batch_run(b, CUTE_BATCH_GRAPH, stream);
        if (s == CUTE_OK) ms = timer.stop_ms();
    }
    for (int i = 0; s == CUTE_OK && i < n_items; i++)
        s = cute_batch_counts(b, i, counts[i], counts_on_device, stream);
    if (s == CUTE_OK && st) {
        s = cute_batch_stats(b, -1, st, stream);
        st->ms_count = ms;
    } else if (s == CUTE_OK) {
        cute_count_stats tmp;
        s = cute_batch_stats(b, -1, &tmp, stream);
    }
    if (s == CUTE_OK) {
        hipError_t e = hipStreamSynchronize(hs);
        if (e != hipSuccess) s = hip_status(e, "hipStreamSynchronize");
    }
    cute_batch_free(b);
    return s;
}
