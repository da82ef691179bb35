// Jackknife pair counts by region decomposition.
//
// With K regions, the jackknife catalog k is the whole catalog without the
// points of region k. Its autocorrelation is the total minus T_k, the pairs
// with at least one point in region k (counted once). One pass gives every
// T_k: over the full stencil (every ordered pair (i, j), i != j, visited once
// from its first point) a pair adds 1 to the home region's histogram when
// both points share the region, 2 otherwise. Region a's histogram then holds
// 2 H_aa + 2 sum_{b != a} H_ab = 2 T_a (H_ab: unordered pairs between
// regions a and b; a same-region pair is visited from both of its points).
// The total is one ordinary autocorrelation. The cost is about three counts
// of the catalog, whatever K, instead of K masked counts.
//
// A cross-correlation (catalogs A and B, each with its regions) works the
// same way with two passes: pairs whose A point lies in region k (A homes,
// weight 1) plus pairs whose B point lies in region k and whose A point does
// not (B homes, A neighbours, weight 0 for a neighbour in the home region and
// 1 otherwise) make T_k, and jack_k = total - T_k. Pair separations are
// symmetric, so a pair counted from its B point lands in the same bin.
//
// A pass runs on a copy of the home grid whose points are sorted by region
// inside each cell (the cells and their offsets are unchanged), so that home
// tiles hold a single region; the tiles of one region form one item of a
// batched launch, whose workgroup histogram then always belongs to one
// region.
#include <hipcub/hipcub.hpp>
#include <string.h>

#include <algorithm>
#include <vector>

#include "cute_internal.h"
#include "runtime.h"

using namespace cute;

namespace {

// key (cell, region) of every sorted point; one thread per cell
__global__ __launch_bounds__(256) void k_region_keys(const uint32_t* __restrict__ cs, uint32_t ncells,
                                                     const P64* __restrict__ p64,
                                                     const int32_t* __restrict__ region,
                                                     uint32_t K, uint64_t* __restrict__ key,
                                                     uint32_t* __restrict__ perm,
                                                     uint32_t* __restrict__ bad) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    for (uint32_t i = cs[c]; i < cs[c + 1]; i++) {
        const int32_t r = region[p64[i].idx];
        if (r < 0 || (uint32_t)r >= K) atomicOr(bad, 1u);
        const uint32_t rr = (r < 0 || (uint32_t)r >= K) ? 0u : (uint32_t)r;
        key[i] = (uint64_t)c * K + rr;
        perm[i] = i;
    }
}

// the grid copy in (cell, region) order, and each point's region
__global__ __launch_bounds__(256) void k_region_gather(uint32_t n, const uint32_t* __restrict__ perm,
                                                       const float4* __restrict__ p32,
                                                       const P64* __restrict__ p64,
                                                       const int32_t* __restrict__ region,
                                                       float4* __restrict__ q32, P64* __restrict__ q64,
                                                       uint16_t* __restrict__ reg) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    const P64 p = p64[j];
    q32[i] = p32[j];
    q64[i] = p;
    reg[i] = (uint16_t)region[p.idx];
}

}  // namespace

namespace {

// A grid copy whose points are in (cell, region) order, in stream-ordered
// temporary memory, with the region of each point.
struct RegionCopy {
    GridHost R;
    uint16_t* regs = nullptr;
};

cute_status region_copy(const GridHost& G, const int32_t* region, int32_t regions_on_device,
                        int32_t K, hipStream_t hs, TempList& tmp, RegionCopy* out) {
    cute_status s;
    const int64_t n = G.n;
    const uint32_t ncells = (uint32_t)((int64_t)G.nx * G.ny * G.nz);
    out->R = G;
    if (n == 0) return CUTE_OK;
    // regions on the device
    const int32_t* dreg = region;
    if (!regions_on_device) {
        int32_t* r = nullptr;
        if ((s = tmp.alloc(&r, (size_t)n)) != CUTE_OK) return s;
        CUTE_HIP(hipMemcpyAsync(r, region, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, hs));
        dreg = r;
    }
    // sort the points of each cell by region
    uint64_t *k0, *k1;
    uint32_t *v0, *v1, *bad;
    if ((s = tmp.alloc(&k0, (size_t)n)) != CUTE_OK) return s;
    if ((s = tmp.alloc(&k1, (size_t)n)) != CUTE_OK) return s;
    if ((s = tmp.alloc(&v0, (size_t)n)) != CUTE_OK) return s;
    if ((s = tmp.alloc(&v1, (size_t)n)) != CUTE_OK) return s;
    if ((s = tmp.alloc(&bad, 1)) != CUTE_OK) return s;
    CUTE_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), hs));
    hipLaunchKernelGGL(k_region_keys, dim3((ncells + 255) / 256), dim3(256), 0, hs, G.cstart,
                       ncells, G.p64, dreg, (uint32_t)K, k0, v0, bad);
    CUTE_HIP(hipGetLastError());
    int bits = 1;
    while (bits < 64 && (((uint64_t)ncells * (uint64_t)K) >> bits) != 0) bits++;
    size_t tb = 0;
    CUTE_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, v0, v1, (int)n, 0, bits, hs));
    unsigned char* tsort = nullptr;
    if ((s = tmp.alloc(&tsort, tb)) != CUTE_OK) return s;
    CUTE_HIP(hipcub::DeviceRadixSort::SortPairs(tsort, tb, k0, k1, v0, v1, (int)n, 0, bits, hs));
    uint32_t hbad = 0;
    CUTE_HIP(hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, hs));
    CUTE_HIP(hipStreamSynchronize(hs));
    if (hbad) return fail(CUTE_E_INVALID_ARG, "region labels must be in [0, K)");
    // the grid copy: same cells, points in (cell, region) order
    GridHost& R = out->R;
    unsigned char* blk = nullptr;
    const size_t b64 = (size_t)n * sizeof(P64), b32 = (size_t)n * sizeof(float4);
    const size_t bcs = ((size_t)ncells + 1) * sizeof(uint32_t);
    if ((s = tmp.alloc(&blk, b64 + b32 + bcs + (size_t)n * sizeof(uint16_t))) != CUTE_OK) return s;
    R.block = blk;
    R.p64 = reinterpret_cast<P64*>(blk);
    R.p32 = reinterpret_cast<float4*>(blk + b64);
    R.cstart = reinterpret_cast<uint32_t*>(blk + b64 + b32);
    out->regs = reinterpret_cast<uint16_t*>(blk + b64 + b32 + bcs);
    CUTE_HIP(hipMemcpyAsync(R.cstart, G.cstart, bcs, hipMemcpyDeviceToDevice, hs));
    hipLaunchKernelGGL(k_region_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, hs,
                       (uint32_t)n, v1, G.p32, G.p64, dreg, R.p32, R.p64, out->regs);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

// One region pass: the region-pure home tiles of `home` against the
// neighbours of `nb` (the full stencil). Item k collects the pairs of the
// region-k home tiles, each weighted wsame when its neighbour's region
// (nb_regs) is k and wdiff otherwise (weight 1 without nb_regs); selfx when
// home and neighbours are one catalog (pairs j != i in the home tile's own
// span). h receives K histograms of nbins; st accumulates the statistics.
cute_status region_pass(const RegionCopy& home, const GridHost& nb, const uint16_t* nb_regs,
                        bool selfx, uint32_t wsame, uint32_t wdiff, int32_t K,
                        const cute_binning* bins, cute_precision prec, hipStream_t hs,
                        std::vector<uint64_t>* h, cute_count_stats* st) {
    cute_status s;
    const GridHost& R = home.R;
    Plan pl;
    plan_binning(bins, pl);
    ItemGeom geo;
    if ((s = plan_item(R, nb, false, bins, pl, &geo)) != CUTE_OK) return s;
    if (selfx && geo.stencil.empty() && R.n > 0)
        return fail(CUTE_E_UNSUPPORTED, "stencil too large for the region pass");
    plan_bands(bins, geo.em, pl);
    if ((s = plan_lds(pl, 16)) != CUTE_OK) return s;
    const int nbins = pl.a.nbins;
    h->assign((size_t)K * nbins, 0);
    if (R.n == 0 || nb.n == 0) return CUTE_OK;
    int dev = 0;
    if ((s = ensure_device_ready(&dev)) != CUTE_OK) return s;
    TempList tmp(hs);
    // region-pure home tiles, grouped by region on the host
    Tile* tiles = nullptr;
    uint32_t ntiles = 0;
    if ((s = build_tiles(R, geo.max_w, hs, &tiles, &ntiles, home.regs)) != CUTE_OK) return s;
    std::vector<Tile> ht(ntiles);
    std::vector<uint16_t> hreg((size_t)R.n);
    hipError_t e = hipMemcpyAsync(ht.data(), tiles, ntiles * sizeof(Tile), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hreg.data(), home.regs, (size_t)R.n * sizeof(uint16_t),
                           hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    dfree(tiles, hs);
    if (e != hipSuccess) return hip_status(e, "region tiles");
    std::vector<uint32_t> off((size_t)K + 1, 0);
    for (const Tile& t : ht) off[hreg[t.start] + 1]++;
    for (int k = 0; k < K; k++) off[k + 1] += off[k];
    std::vector<Tile> grouped(ntiles);
    {
        std::vector<uint32_t> at(off.begin(), off.end() - 1);
        for (const Tile& t : ht) grouped[at[hreg[t.start]]++] = t;
    }
    // device buffers of the launch: tables, stencil, tiles, items, chunks, histograms
    Tile* dtiles;
    double *dT1, *dT2;
    float2 *dB1, *dB2;
    int4* dst;
    CountArgs* dargs;
    unsigned long long* work;  // K * nbins histograms, 4 stats per item, chunk head
    if ((s = tmp.alloc(&dtiles, std::max<size_t>(ntiles, 1))) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dT1, pl.T1.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dT2, pl.T2.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dB1, pl.band1.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dB2, pl.band2.size())) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dst, std::max<size_t>(geo.stencil.size(), 1))) != CUTE_OK) return s;
    if ((s = tmp.alloc(&dargs, (size_t)K)) != CUTE_OK) return s;
    const size_t wwords = (size_t)K * nbins + 4 * (size_t)K + 1;
    if ((s = tmp.alloc(&work, wwords)) != CUTE_OK) return s;
    if (ntiles)
        CUTE_HIP(hipMemcpyAsync(dtiles, grouped.data(), ntiles * sizeof(Tile), hipMemcpyHostToDevice,
                                hs));
    CUTE_HIP(hipMemcpyAsync(dT1, pl.T1.data(), pl.T1.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dT2, pl.T2.data(), pl.T2.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dB1, pl.band1.data(), pl.band1.size() * 8, hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemcpyAsync(dB2, pl.band2.data(), pl.band2.size() * 8, hipMemcpyHostToDevice, hs));
    if (!geo.stencil.empty())
        CUTE_HIP(hipMemcpyAsync(dst, geo.stencil.data(), geo.stencil.size() * sizeof(int4),
                                hipMemcpyHostToDevice, hs));
    CUTE_HIP(hipMemsetAsync(work, 0, wwords * 8, hs));
    std::vector<CountArgs> args((size_t)K);
    for (int k = 0; k < K; k++) {
        CountArgs& a = args[k];
        a = pl.a;
        apply_item(geo, &a);
        a.self = dargs + k;
        a.T1 = dT1;
        a.T2 = dT2;
        a.band1 = dB1;
        a.band2 = dB2;
        a.stencil = geo.stencil.empty() ? nullptr : dst;
        a.nst = (int)geo.stencil.size();
        a.tiles = dtiles + off[k];
        a.ntiles = off[k + 1] - off[k];
        a.counts = work + (size_t)k * nbins;
        a.stats = work + (size_t)K * nbins + 4 * (size_t)k;
        a.regs = nb_regs;
        a.region = k;
        a.wsame = wsame;
        a.wdiff = wdiff;
        a.selfx = selfx ? 1 : 0;
    }
    CUTE_HIP(hipMemcpyAsync(dargs, args.data(), sizeof(CountArgs) * (size_t)K, hipMemcpyHostToDevice,
                            hs));
    // chunks: runs of up to 64 tiles of one region, regions in order
    int per_cu = 1, ncu = 0;
    if ((s = batch_prepare(pl.mode, (int)prec, pl.est, pl.lds, &per_cu)) != CUTE_OK) return s;
    CUTE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t grid_max = (uint64_t)per_cu * ncu;
    uint64_t per = ntiles / std::max<uint64_t>(grid_max * 8, 1);
    per = std::max<uint64_t>(4, std::min<uint64_t>(64, per));
    std::vector<uint32_t> ch;
    for (int k = 0; k < K; k++)
        for (uint32_t t0 = 0; t0 < off[k + 1] - off[k]; t0 += (uint32_t)per) {
            ch.push_back((uint32_t)k);
            ch.push_back(t0);
            ch.push_back(std::min<uint32_t>(t0 + (uint32_t)per, off[k + 1] - off[k]));
            ch.push_back(0u);
        }
    const uint32_t nch = (uint32_t)(ch.size() / 4);
    uint32_t* dch = nullptr;
    if ((s = tmp.alloc(&dch, std::max<size_t>(ch.size(), 4))) != CUTE_OK) return s;
    if (nch) CUTE_HIP(hipMemcpyAsync(dch, ch.data(), ch.size() * 4, hipMemcpyHostToDevice, hs));
    BatchArgs ba;
    memset(&ba, 0, sizeof(ba));
    ba.items = dargs;
    ba.chunks = dch;
    ba.nchunks = nch;
    ba.head = reinterpret_cast<uint32_t*>(work + (size_t)K * nbins + 4 * (size_t)K);
    ba.n1 = pl.a.n1;
    ba.n2 = pl.a.n2;
    ba.nbins = nbins;
    ba.copies = pl.a.copies;
    ba.hist_words = pl.a.hist_words;
    ba.T1 = dT1;
    ba.T2 = dT2;
    ba.band1 = dB1;
    ba.band2 = dB2;
    double ms = 0.0;
    if (nch) {
        EventTimer timer(hs);
        const int gsz = (int)std::min<uint64_t>(grid_max, nch);
        if ((s = batch_launch(ba, pl.mode, (int)prec, pl.est, gsz, pl.lds, hs)) != CUTE_OK) return s;
        timer.stop();
        ms = timer.elapsed_ms();
    }
    std::vector<unsigned long long> hw(wwords);
    CUTE_HIP(hipMemcpyAsync(hw.data(), work, wwords * 8, hipMemcpyDeviceToHost, hs));
    CUTE_HIP(hipStreamSynchronize(hs));
    uint64_t tiles_done = 0;
    for (int k = 0; k < K; k++) {
        const unsigned long long* sv = hw.data() + (size_t)K * nbins + 4 * (size_t)k;
        st->pair_evals += sv[0];
        st->retests += sv[1];
        st->flips += sv[2];
        tiles_done += sv[3];
    }
    st->tiles += tiles_done;
    st->ms_count += ms;
    if (tiles_done != ntiles) return fail(CUTE_E_INTERNAL, "not every region tile was processed");
    for (size_t i = 0; i < h->size(); i++) (*h)[i] = hw[i];
    return CUTE_OK;
}

cute_status check_common(const cute_grid* g, const int32_t* region, int32_t K,
                         const cute_binning* bins, cute_precision prec) {
    // every argument is checked before the grid is read
    if (!g || !region) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    if (K < 1 || K > 65535) return fail(CUTE_E_INVALID_ARG, "K must be in [1, 65535]");
    cute_status s = validate_binning(bins);
    if (s != CUTE_OK) return s;
    if (prec != CUTE_PREC_FP64 && prec != CUTE_PREC_FP32_EDGE && prec != CUTE_PREC_FP32_ONLY)
        return fail(CUTE_E_INVALID_ARG, "unknown precision");
    if (g->h.wt != nullptr) return fail(CUTE_E_UNSUPPORTED, "pixel maps have no jackknife pass");
    if (g->h.geom == CUTE_GEOM_SPHERE) return fail(CUTE_E_UNSUPPORTED, "jackknife regions need a 3-D grid");
    return CUTE_OK;
}

void add_stats(cute_count_stats* st, const cute_count_stats& a, const cute_count_stats& b) {
    if (!st) return;
    *st = a;
    st->pair_evals += b.pair_evals;
    st->retests += b.retests;
    st->flips += b.flips;
    st->tiles += b.tiles;
    st->ms_count += b.ms_count;
}

}  // namespace

extern "C" cute_status cute_count_jackknife(const cute_grid* grid, const int32_t* region,
                                            int32_t regions_on_device, int32_t K,
                                            const cute_binning* bins, cute_precision prec,
                                            uint64_t* total, uint64_t* jack,
                                            cute_count_stats* st, void* stream) {
    if (!total || !jack) return fail(CUTE_E_INVALID_ARG, "NULL argument");
    cute_status s = check_common(grid, region, K, bins, prec);
    if (s != CUTE_OK) return s;
    const GridHost& G = grid->h;
    hipStream_t hs = (hipStream_t)stream;
    // the total: one ordinary autocorrelation
    cute_count_stats st_tot, st_reg;
    memset(&st_tot, 0, sizeof(st_tot));
    memset(&st_reg, 0, sizeof(st_reg));
    if ((s = cute_count_pairs(grid, nullptr, bins, prec, total, 0, &st_tot, stream)) != CUTE_OK)
        return s;
    const int nbins = bins->n1 * (bins->n2 > 0 ? bins->n2 : 1);
    std::vector<uint64_t> h2((size_t)K * nbins, 0);
    if (G.n > 0) {
        TempList tmp(hs);
        RegionCopy rc;
        if ((s = region_copy(G, region, regions_on_device, K, hs, tmp, &rc)) != CUTE_OK) return s;
        if ((s = region_pass(rc, rc.R, rc.regs, true, 1u, 2u, K, bins, prec, hs, &h2, &st_reg)) !=
            CUTE_OK)
            return s;
    }
    // jack_k = total - T_k, T_k = (region k's weighted histogram) / 2
    for (int k = 0; k < K; k++)
        for (int b = 0; b < nbins; b++) {
            const uint64_t w = h2[(size_t)k * nbins + b];
            const uint64_t t = w / 2;
            if ((w & 1u) || t > total[b])
                return fail(CUTE_E_INTERNAL, "region histograms are inconsistent");
            jack[(size_t)k * nbins + b] = total[b] - t;
        }
    add_stats(st, st_tot, st_reg);
    return CUTE_OK;
}

extern "C" cute_status cute_count_jackknife_cross(const cute_grid* a, const int32_t* region_a,
                                                  const cute_grid* b, const int32_t* region_b,
                                                  int32_t regions_on_device, int32_t K,
                                                  const cute_binning* bins, cute_precision prec,
                                                  uint64_t* total, uint64_t* jack,
                                                  cute_count_stats* st, void* stream) {
    if (!total || !jack || !a || !region_a || !b || !region_b)
        return fail(CUTE_E_INVALID_ARG, "NULL argument");
    if (K < 1 || K > 65535) return fail(CUTE_E_INVALID_ARG, "K must be in [1, 65535]");
    cute_status s = check_common(a, region_a, K, bins, prec);
    if (s != CUTE_OK) return s;
    if ((s = check_common(b, region_b, K, bins, prec)) != CUTE_OK) return s;
    if (a == b) return fail(CUTE_E_INVALID_ARG, "a and b are one grid: use cute_count_jackknife");
    hipStream_t hs = (hipStream_t)stream;
    cute_count_stats st_tot, st_reg;
    memset(&st_tot, 0, sizeof(st_tot));
    memset(&st_reg, 0, sizeof(st_reg));
    if ((s = cute_count_pairs(a, b, bins, prec, total, 0, &st_tot, stream)) != CUTE_OK) return s;
    const int nbins = bins->n1 * (bins->n2 > 0 ? bins->n2 : 1);
    std::vector<uint64_t> ha((size_t)K * nbins, 0), hb((size_t)K * nbins, 0);
    if (a->h.n > 0 && b->h.n > 0) {
        TempList tmp(hs);
        RegionCopy ra, rb;
        if ((s = region_copy(a->h, region_a, regions_on_device, K, hs, tmp, &ra)) != CUTE_OK) return s;
        if ((s = region_copy(b->h, region_b, regions_on_device, K, hs, tmp, &rb)) != CUTE_OK) return s;
        // pairs whose A point lies in region k
        if ((s = region_pass(ra, b->h, nullptr, false, 1u, 1u, K, bins, prec, hs, &ha, &st_reg)) !=
            CUTE_OK)
            return s;
        // pairs whose B point lies in region k and whose A point does not
        if ((s = region_pass(rb, ra.R, ra.regs, false, 0u, 1u, K, bins, prec, hs, &hb, &st_reg)) !=
            CUTE_OK)
            return s;
    }
    for (int k = 0; k < K; k++)
        for (int c = 0; c < nbins; c++) {
            const size_t i = (size_t)k * nbins + c;
            const uint64_t t = ha[i] + hb[i];
            if (t > total[c]) return fail(CUTE_E_INTERNAL, "region histograms are inconsistent");
            jack[i] = total[c] - t;
        }
    add_stats(st, st_tot, st_reg);
    return CUTE_OK;
}
