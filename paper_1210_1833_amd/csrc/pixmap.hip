// Pixel maps for the pixelised angular correlation (Sec. 3.4, angular
// correlation function): the objects of a catalog on the unit sphere are
// binned into equal-area pixels, and each non-empty pixel becomes one point
// at its centre that carries its occupancy as a weight. Counting pixel pairs
// with weight n_p n_q then stands in for counting object pairs, with every
// object moved to the centre of its pixel.
//
// Pixels are cells in (cos theta, phi), as in the pixelisation of Sec. 3.3:
// n_cth rings of equal width in cos theta = z and n_phi sectors of equal width
// in phi. Ring and sector are integers decided in FP64 by fixed rules (the
// comments of cute_build_pixel_map in the public header state them), so that
// any FP64 implementation of the rules finds the same pixel:
//  - ring = floor((z + 1) * (n_cth / 2)), clamped to [0, n_cth - 1];
//  - sector: the k whose boundary rays enclose the point, "on or
//    counter-clockwise of the ray (c, s)" being fl(fl(y c) - fl(x s)) >= 0,
//    with (c, s) = (cos, sin) of fl(fl(2 pi k) / n_phi) from the C library;
//    the search starts at the sector of atan2 and steps to the enclosing one.
// The ray and centre tables are computed on the host with the C library's
// cos and sin; the kernels only multiply and compare.
#include <hipcub/hipcub.hpp>
#include <math.h>
#include <string.h>

#include <vector>

#include "cute_internal.h"
#include "runtime.h"

using namespace cute;

namespace {

constexpr int kPB = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// ring * n_phi + sector of every point; bad[0]: non-finite or non-unit input,
// bad[1]: a sector search that did not settle
__global__ __launch_bounds__(kPB) void k_pixel_ids(const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z, int64_t n,
                                                   int n_cth, int n_phi,
                                                   const double2* __restrict__ ray,
                                                   uint32_t* __restrict__ ids,
                                                   uint32_t* __restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)kPB + threadIdx.x;
    if (i >= n) return;
    const double px = x[i], py = y[i], pz = z[i];
    const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
    const double n2 = px * px + py * py + pz * pz;
    if (!fin || fabs(n2 - 1.0) > 1e-6) {
        atomicOr(&bad[0], 1u);
        ids[i] = 0u;
        return;
    }
    const double t = (pz + 1.0) * (0.5 * (double)n_cth);
    int r = (int)floor(t);
    r = r < 0 ? 0 : (r > n_cth - 1 ? n_cth - 1 : r);
    int k = 0;
    if (px * px + py * py != 0.0) {
        double f = atan2(py, px);
        if (f < 0.0) f += kTwoPi;
        k = (int)floor(f / kTwoPi * (double)n_phi);
        k = k < 0 ? 0 : (k > n_phi - 1 ? n_phi - 1 : k);
        bool found = false;
        for (int it = 0; it < 4 && !found; it++) {
            const int k1 = k + 1 == n_phi ? 0 : k + 1;
            const double2 a = ray[k], b = ray[k1];
            const double sa = py * a.x - px * a.y;
            const double sb = py * b.x - px * b.y;
            if (sa < 0.0) k = k == 0 ? n_phi - 1 : k - 1;
            else if (sb >= 0.0) k = k1;
            else found = true;
        }
        if (!found) atomicOr(&bad[1], 1u);
    }
    ids[i] = (uint32_t)r * (uint32_t)n_phi + (uint32_t)k;
}

// centre of each pixel: (s_r cos f_k, s_r sin f_k, c_r) from the host tables
// ring[r] = (c_r, s_r) and sec[k] = (cos f_k, sin f_k)
__global__ __launch_bounds__(kPB) void k_pixel_centres(const uint32_t* __restrict__ ids, int64_t m,
                                                       int n_phi, const double2* __restrict__ ring,
                                                       const double2* __restrict__ sec,
                                                       double* __restrict__ x, double* __restrict__ y,
                                                       double* __restrict__ z) {
    const int64_t i = blockIdx.x * (int64_t)kPB + threadIdx.x;
    if (i >= m) return;
    const uint32_t id = ids[i];
    const double2 rc = ring[id / (uint32_t)n_phi];
    const double2 sc = sec[id % (uint32_t)n_phi];
    x[i] = rc.y * sc.x;
    y[i] = rc.y * sc.y;
    z[i] = rc.x;
}

// occupancy of each sorted grid point (the grid keeps the input index)
__global__ __launch_bounds__(kPB) void k_gather_weights(const P64* __restrict__ p64, int64_t m,
                                                        const uint32_t* __restrict__ cnt,
                                                        uint32_t* __restrict__ wt) {
    const int64_t i = blockIdx.x * (int64_t)kPB + threadIdx.x;
    if (i >= m) return;
    wt[i] = cnt[p64[i].idx];
}

// sum over points of w (w - 1) / 2, the object pairs that share a pixel (at
// zero separation), added to one count
__global__ __launch_bounds__(kPB) void k_pixel_self_pairs(const uint32_t* __restrict__ w, int64_t m,
                                                          unsigned long long* __restrict__ bin) {
    __shared__ unsigned long long part[kPB / 64];
    unsigned long long s = 0;
    for (int64_t i = blockIdx.x * (int64_t)kPB + threadIdx.x; i < m; i += (int64_t)gridDim.x * kPB) {
        const uint64_t v = w[i];
        s += v * (v - (v > 0u ? 1u : 0u)) / 2u;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kPB / 64; k++) t += part[k];
        if (t) atomicAdd(bin, t);
    }
}

}  // namespace

namespace cute {

cute_status add_pixel_self_pairs(const GridHost& g, unsigned long long* bin, hipStream_t s) {
    if (g.wt == nullptr || g.n == 0) return CUTE_OK;
    const int64_t nb = std::min<int64_t>(1024, (g.n + kPB - 1) / kPB);
    hipLaunchKernelGGL(k_pixel_self_pairs, dim3((unsigned)nb), dim3(kPB), 0, s, g.wt, g.n, bin);
    CUTE_HIP(hipGetLastError());
    return CUTE_OK;
}

}  // namespace cute

extern "C" cute_status cute_build_pixel_map(const double* x, const double* y, const double* z,
                                            int64_t n, int32_t n_cth, int32_t n_phi,
                                            const cute_grid_params* p, void* stream,
                                            cute_grid** out) {
    if (!out) return fail(CUTE_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(CUTE_E_INVALID_ARG, "params is NULL");
    if (p->geom != CUTE_GEOM_SPHERE) return fail(CUTE_E_INVALID_ARG, "pixel maps need the SPHERE geometry");
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CUTE_E_INVALID_ARG, "n must be in [0, 2^31)");
    if (n > 0 && (!x || !y || !z)) return fail(CUTE_E_INVALID_ARG, "coordinate pointer is NULL");
    if (n_cth < 1 || n_phi < 8 || (int64_t)n_cth * n_phi >= (int64_t(1) << 31))
        return fail(CUTE_E_INVALID_ARG, "need n_cth >= 1, n_phi >= 8, n_cth * n_phi < 2^31");
    int dev = 0;
    cute_status st = ensure_device_ready(&dev);
    if (st != CUTE_OK) return st;
    hipStream_t s = (hipStream_t)stream;
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

    // host tables: boundary rays, ring centres, sector centres
    std::vector<double2> h_tab((size_t)2 * n_phi + n_cth);
    for (int k = 0; k < n_phi; k++) {
        const double a = kTwoPi * (double)k / (double)n_phi;
        h_tab[k] = make_double2(cos(a), sin(a));
        const double f = kTwoPi * ((double)k + 0.5) / (double)n_phi;
        h_tab[(size_t)n_phi + k] = make_double2(cos(f), sin(f));
    }
    for (int r = 0; r < n_cth; r++) {
        const double c = (double)(2 * r + 1) / (double)n_cth - 1.0;
        h_tab[(size_t)2 * n_phi + r] = make_double2(c, sqrt((1.0 - c) * (1.0 + c)));
    }
    double2* d_tab = nullptr;
    if ((st = tmp.alloc(&d_tab, h_tab.size())) != CUTE_OK) return st;
    CUTE_HIP(hipMemcpyAsync(d_tab, h_tab.data(), h_tab.size() * sizeof(double2),
                            hipMemcpyHostToDevice, s));
    const double2* d_ray = d_tab;
    const double2* d_sec = d_tab + n_phi;
    const double2* d_ring = d_tab + 2 * (size_t)n_phi;

    // pixel ids, sorted, run-length encoded into (id, occupancy)
    uint32_t *ids = nullptr, *ids2 = nullptr, *uniq = nullptr, *cnt = nullptr, *aux = nullptr;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    if ((st = tmp.alloc(&ids, nn)) != CUTE_OK) return st;
    if ((st = tmp.alloc(&ids2, nn)) != CUTE_OK) return st;
    if ((st = tmp.alloc(&uniq, nn)) != CUTE_OK) return st;
    if ((st = tmp.alloc(&cnt, nn)) != CUTE_OK) return st;
    if ((st = tmp.alloc(&aux, 4)) != CUTE_OK) return st;  // bad[2], runs, pad
    CUTE_HIP(hipMemsetAsync(aux, 0, 4 * sizeof(uint32_t), s));
    if (n > 0) {
        hipLaunchKernelGGL(k_pixel_ids, dim3((unsigned)((n + kPB - 1) / kPB)), dim3(kPB), 0, s, dx,
                           dy, dz, n, (int)n_cth, (int)n_phi, d_ray, ids, aux);
        CUTE_HIP(hipGetLastError());
        int bits = 1;
        while (bits < 32 && (((uint64_t)n_cth * (uint64_t)n_phi - 1u) >> bits) != 0) bits++;
        size_t tb = 0, tb2 = 0;
        CUTE_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, ids, ids2, (int)n, 0, bits, s));
        CUTE_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb2, ids2, uniq, cnt, aux + 2, (int)n, s));
        unsigned char* tstore = nullptr;
        if ((st = tmp.alloc(&tstore, std::max(tb, tb2))) != CUTE_OK) return st;
        CUTE_HIP(hipcub::DeviceRadixSort::SortKeys(tstore, tb, ids, ids2, (int)n, 0, bits, s));
        CUTE_HIP(hipcub::DeviceRunLengthEncode::Encode(tstore, tb2, ids2, uniq, cnt, aux + 2, (int)n, s));
    }
    uint32_t haux[4] = {0, 0, 0, 0};
    CUTE_HIP(hipMemcpyAsync(haux, aux, sizeof(haux), hipMemcpyDeviceToHost, s));
    CUTE_HIP(hipStreamSynchronize(s));
    if (haux[0]) return fail(CUTE_E_INVALID_ARG, "pixel maps need finite unit vectors");
    if (haux[1]) return fail(CUTE_E_INTERNAL, "pixel sector search did not settle");
    const int64_t m = n > 0 ? (int64_t)haux[2] : 0;

    // the centres, gridded like any angular catalog
    double* cxyz = nullptr;
    if ((st = tmp.alloc(&cxyz, 3 * (size_t)(m > 0 ? m : 1))) != CUTE_OK) return st;
    if (m > 0) {
        hipLaunchKernelGGL(k_pixel_centres, dim3((unsigned)((m + kPB - 1) / kPB)), dim3(kPB), 0, s,
                           uniq, m, (int)n_phi, d_ring, d_sec, cxyz, cxyz + m, cxyz + 2 * m);
        CUTE_HIP(hipGetLastError());
    }
    cute_grid_params gp = *p;
    gp.device_ptrs = 1;
    cute_grid* g = nullptr;
    if ((st = cute_build_grid(cxyz, cxyz + m, cxyz + 2 * m, m, &gp, stream, &g)) != CUTE_OK) return st;

    // [wt | pix_id | pix_n], owned by the grid
    uint32_t* wb = nullptr;
    if ((st = dalloc(&wb, 3 * (size_t)(m > 0 ? m : 1), s)) != CUTE_OK) {
        cute_free_grid(g);
        return st;
    }
    GridHost& G = g->h;
    G.wblock = wb;
    G.wt = wb;
    G.pix_id = wb + m;
    G.pix_n = wb + 2 * m;
    G.n_cth = n_cth;
    G.n_phi = n_phi;
    if (m > 0) {
        hipError_t e = hipMemcpyAsync(G.pix_id, uniq, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(G.pix_n, cnt, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gather_weights, dim3((unsigned)((m + kPB - 1) / kPB)), dim3(kPB), 0,
                               s, G.p64, m, cnt, G.wt);
            e = hipGetLastError();
        }
        if (e != hipSuccess) {
            cute_free_grid(g);
            return hip_status(e, "pixel map weights");
        }
    }
    timer.stop();
    const hipError_t we = timer.b ? hipEventSynchronize(timer.b) : hipStreamSynchronize(s);
    if (we != hipSuccess) {
        cute_free_grid(g);
        return fail(CUTE_E_DEVICE, "pixel map sync");
    }
    G.ms_build = timer.elapsed_ms();
    // the whole map is built: its time replaces that of the centres' grid
    if (G.ev_ready) (void)hipEventDestroy(G.ev_ready);
    if (G.ev_start) (void)hipEventDestroy(G.ev_start);
    G.ev_ready = G.ev_start = nullptr;
    *out = g;
    return CUTE_OK;
}

extern "C" cute_status cute_pixel_map_read(const cute_grid* g, uint32_t* ids, uint32_t* counts,
                                           void* stream) {
    if (!g) return fail(CUTE_E_INVALID_ARG, "grid is NULL");
    const GridHost& G = g->h;
    if (G.wt == nullptr) return fail(CUTE_E_INVALID_ARG, "not a pixel map");
    hipStream_t s = (hipStream_t)stream;
    cute_status st = grid_wait(g, s);
    if (st != CUTE_OK) return st;
    if (G.n > 0 && ids)
        CUTE_HIP(hipMemcpyAsync(ids, G.pix_id, G.n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (G.n > 0 && counts)
        CUTE_HIP(hipMemcpyAsync(counts, G.pix_n, G.n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CUTE_HIP(hipStreamSynchronize(s));
    return CUTE_OK;
}
