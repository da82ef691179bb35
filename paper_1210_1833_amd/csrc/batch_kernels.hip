// Batched pair counts: many (grid, grid, mask) items that share one binning in
// one persistent launch.
//
// Work is handed out in chunks (a run of home tiles of one item) to whole
// workgroups: the four waves of a workgroup take the chunk's tiles one at a
// time from an LDS counter, so the shared 64-bit LDS histogram always holds
// counts of a single item. When a workgroup moves to a chunk of another item
// it first sums its histogram into that item's global counts. Chunks are
// ordered by the estimated cost of their item, largest first, so that the
// small items fill the tail of the launch. Point masks (bits in sorted order)
// leave excluded home points and neighbour lanes idle.
#include <type_traits>

#include "count_device.h"

namespace cute {

namespace {

typedef const __attribute__((address_space(4))) CountArgs* cargp;

// Sum the workgroup's histogram copies into counts (one atomic per non-empty
// bin) and clear them (counters of 4 bytes when H32, else 8).
template <bool H32>
__device__ void flush_hist(unsigned char* hist0, int nbins, int copies, unsigned long long* counts) {
    typedef typename std::conditional<H32, uint32_t, unsigned long long>::type word;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        uint64_t s = 0;
        word* hh = reinterpret_cast<word*>(hist0) + (size_t)b * copies;
        for (int c = 0; c < copies; c++) {
            s += hh[c];
            hh[c] = 0;
        }
        if (s) atomicAdd(&counts[b], (unsigned long long)s);
    }
}

template <int MODE, int PREC, int EST>
__global__ __launch_bounds__(256, (kWgPerCu<MODE, PREC>)) void k_count_batch(BatchArgs BA) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int n1 = BA.n1, n2 = BA.n2;
    const int n2p = n2 > 0 ? n2 : 0;
    double* T1 = reinterpret_cast<double*>(smem);
    double* T2 = T1 + (n1 + 1);
    float2* B1 = reinterpret_cast<float2*>(T2 + (n2p + 1));
    float2* B2 = B1 + n1;
    constexpr bool H32 = kH32<MODE>;
    // the histogram: hist_words counters of 4 (kH32) or 8 bytes, padded to 8
    unsigned char* hist0 = reinterpret_cast<unsigned char*>(B2 + (n2p > 0 ? n2p : 1));
    const size_t hbytes = ((size_t)BA.hist_words * (H32 ? 4 : 8) + 7) & ~(size_t)7;
    uint32_t* q0 = reinterpret_cast<uint32_t*>(hist0 + hbytes);
    unsigned long long* rs0 = reinterpret_cast<unsigned long long*>(q0 + (size_t)nwaves * 3 * kQCap);
    uint32_t* sp0 = reinterpret_cast<uint32_t*>(rs0 + 2 * nwaves);
    uint32_t* ctl = sp0 + (size_t)nwaves * 3 * kSpanCap;  // chunk id, item, next tile, end tile
    uint32_t* budget = ctl + 4;                           // 32-bit histograms only
    for (int i = threadIdx.x; i <= n1; i += blockDim.x) T1[i] = BA.T1[i];
    for (int i = threadIdx.x; i <= n2p; i += blockDim.x) T2[i] = n2p ? BA.T2[i] : 0.0;
    if (PREC != P_FP64) {
        for (int i = threadIdx.x; i < n1; i += blockDim.x) B1[i] = BA.band1[i];
        for (int i = threadIdx.x; i < n2p; i += blockDim.x) B2[i] = BA.band2[i];
    }
    for (size_t i = threadIdx.x; i < hbytes / 4; i += blockDim.x) reinterpret_cast<uint32_t*>(hist0)[i] = 0u;
    for (int i = threadIdx.x; i < 2 * nwaves; i += blockDim.x) rs0[i] = 0ull;
    if (H32 && threadIdx.x == 0) *budget = 0u;

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

    uint32_t cur = 0xffffffffu;  // item whose counts the histogram holds
    for (;;) {
        __syncthreads();  // every wave is done with the previous chunk
        if (threadIdx.x == 0) {
            const uint32_t c = atomicAdd(BA.head, 1u);
            ctl[0] = c;
            if (c < BA.nchunks) {
                const cu32p ch = (cu32p)(const void*)BA.chunks;
                ctl[1] = ch[4 * c];
                ctl[2] = ch[4 * c + 1];
                ctl[3] = ch[4 * c + 2];
            }
        }
        __syncthreads();
        const uint32_t c = uni(ctl[0]);
        if (c >= BA.nchunks) break;
        const uint32_t item = uni(ctl[1]);
        const uint32_t tend = uni(ctl[3]);
        if (item != cur) {
            if (cur != 0xffffffffu) {
                const CountArgs& Pc = *(const CountArgs*)(cargp)(const void*)(BA.items + cur);
                flush_hist<H32>(hist0, BA.nbins, BA.copies, Pc.counts);
                if (H32 && threadIdx.x == 0) *budget = 0u;
                __syncthreads();
            }
            cur = item;
        }
        const CountArgs& P = *(const CountArgs*)(cargp)(const void*)(BA.items + item);
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&ctl[2], 1u);
            t = uni(t);
            if (t >= tend) break;
            const cu32p tp = (cu32p)(const void*)P.tiles;
            Tile tl;
            tl.start = uni(tp[4 * t]);
            tl.end = uni(tp[4 * t + 1]);
            tl.row = uni(tp[4 * t + 2]);
            tl.c0c1 = uni(tp[4 * t + 3]);
            do_tile<MODE, PREC, EST, true, false>(P, W, S, B1, B2, T1, T2, lane, tl);
        }
        // the re-test queue refers to this item's points: empty it now
        if constexpr (PREC == P_FP32E)
            W.tail = drain_queue<MODE, EST>(P.self, W.hist, W.qi, W.qj, W.qc, W.rstat, B1, B2, T1, T2,
                                            lane, W.tail, true);
        if (lane == 0) {
            atomicAdd(&P.stats[0], (unsigned long long)W.evals);
            atomicAdd(&P.stats[1], W.rstat[0]);
            atomicAdd(&P.stats[2], W.rstat[1]);
            atomicAdd(&P.stats[3], (unsigned long long)W.tiles);
            W.rstat[0] = 0ull;
            W.rstat[1] = 0ull;
        }
        W.evals = W.tiles = 0;
    }
    if (cur != 0xffffffffu) {
        const CountArgs& Pc = *(const CountArgs*)(cargp)(const void*)(BA.items + cur);
        flush_hist<H32>(hist0, BA.nbins, BA.copies, Pc.counts);
    }
}

// Sorted-order exclusion bits of a mask given in the caller's input order:
// bit i of word i / 32 is set when mask[idx of sorted point i] != 0.
__global__ __launch_bounds__(256) void k_mask_bits(const uint8_t* __restrict__ mask,
                                                   const P64* __restrict__ p64, uint32_t n,
                                                   uint32_t* __restrict__ bits) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if ((uint64_t)w * 32u >= n) return;
    uint32_t b = 0;
    for (uint32_t k = 0; k < 32u; k++) {
        const uint32_t i = w * 32u + k;
        if (i < n && mask[p64[i].idx] != 0) b |= 1u << k;
    }
    bits[w] = b;
}

// Zero n 64-bit words (a kernel, so that captured graphs hold no memset).
__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <int MODE, int PREC, int EST>
cute_status prep_one(size_t lds, int* per_cu) {
    auto kern = k_count_batch<MODE, PREC, EST>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_status(e, "hipFuncSetAttribute");
    }
    CUTE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, 64 * kWgWaves, lds));
    if (*per_cu < 1) *per_cu = 1;
    return CUTE_OK;
}

template <int MODE, int PREC, int EST>
cute_status launch_b(const BatchArgs& ba, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_count_batch<MODE, PREC, EST>), dim3(grid), dim3(64 * kWgWaves), lds, s, ba);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

// Dispatch on (mode, prec, est) to F<MODE, PREC, EST>(args...).
#define CUTE_DISPATCH(FN, mode, prec, est, ...)                                              \
    do {                                                                                      \
        const int m_ = (mode), p_ = (prec), e_ = (est) & E_LOG;                               \
        if (m_ == M_RMU_Z && p_ == P_FP32E && est_muf(est)) {                                 \
            if (e_) return FN<1, 1, E_LOG | E_MUF>(__VA_ARGS__);                                \
            return FN<1, 1, E_MUF>(__VA_ARGS__);                                               \
        }                                                                                     \
        switch (m_ * 6 + p_ * 2 + e_) {                                                       \
            case 0: return FN<0, 0, 0>(__VA_ARGS__);                                          \
            case 1: return FN<0, 0, 1>(__VA_ARGS__);                                          \
            case 2: return FN<0, 1, 0>(__VA_ARGS__);                                          \
            case 3: return FN<0, 1, 1>(__VA_ARGS__);                                          \
            case 4: return FN<0, 2, 0>(__VA_ARGS__);                                          \
            case 5: return FN<0, 2, 1>(__VA_ARGS__);                                          \
            case 6: return FN<1, 0, 0>(__VA_ARGS__);                                          \
            case 7: return FN<1, 0, 1>(__VA_ARGS__);                                          \
            case 8: return FN<1, 1, 0>(__VA_ARGS__);                                          \
            case 9: return FN<1, 1, 1>(__VA_ARGS__);                                          \
            case 10: return FN<1, 2, 0>(__VA_ARGS__);                                         \
            case 11: return FN<1, 2, 1>(__VA_ARGS__);                                         \
            case 12: return FN<2, 0, 0>(__VA_ARGS__);                                         \
            case 13: return FN<2, 0, 1>(__VA_ARGS__);                                         \
            case 14: return FN<2, 1, 0>(__VA_ARGS__);                                         \
            case 15: return FN<2, 1, 1>(__VA_ARGS__);                                         \
            case 16: return FN<2, 2, 0>(__VA_ARGS__);                                         \
            case 17: return FN<2, 2, 1>(__VA_ARGS__);                                         \
            case 18: return FN<3, 0, 0>(__VA_ARGS__);                                         \
            case 19: return FN<3, 0, 1>(__VA_ARGS__);                                         \
            case 20: return FN<3, 1, 0>(__VA_ARGS__);                                         \
            case 21: return FN<3, 1, 1>(__VA_ARGS__);                                         \
            case 22: return FN<3, 2, 0>(__VA_ARGS__);                                         \
            case 23: return FN<3, 2, 1>(__VA_ARGS__);                                         \
            case 24: return FN<4, 0, 0>(__VA_ARGS__);                                         \
            case 25: return FN<4, 0, 1>(__VA_ARGS__);                                         \
            case 26: return FN<4, 1, 0>(__VA_ARGS__);                                         \
            case 27: return FN<4, 1, 1>(__VA_ARGS__);                                         \
            case 28: return FN<4, 2, 0>(__VA_ARGS__);                                         \
            case 29: return FN<4, 2, 1>(__VA_ARGS__);                                         \
            default: return fail(CUTE_E_INTERNAL, "unknown kernel variant");                  \
        }                                                                                     \
    } while (0)

}  // namespace

cute_status batch_prepare(int mode, int prec, int est, size_t lds, int* per_cu) {
    CUTE_DISPATCH(prep_one, mode, prec, est, lds, per_cu);
}

cute_status batch_launch(const BatchArgs& ba, int mode, int prec, int est, int grid, size_t lds,
                         hipStream_t s) {
    CUTE_DISPATCH(launch_b, mode, prec, est, ba, grid, lds, s);
}

cute_status mask_bits(const uint8_t* mask, const GridHost& g, uint32_t* bits, hipStream_t s) {
    const uint32_t words = (uint32_t)((g.n + 31) / 32);
    if (words == 0) return CUTE_OK;
    hipLaunchKernelGGL(k_mask_bits, dim3((words + 255) / 256), dim3(256), 0, s, mask, g.p64,
                       (uint32_t)g.n, bits);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

cute_status zero_u64(unsigned long long* p, size_t n, hipStream_t s) {
    if (n == 0) return CUTE_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

cute_status zero_u32(uint32_t* p, size_t n, hipStream_t s) {
    if (n == 0) return CUTE_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

}  // namespace cute
