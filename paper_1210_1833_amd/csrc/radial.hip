// Per-point values in a grid's sorted order, for the radial correlation
// (Sec. 2.1, radial 2PCF; Sec. 3.4): the redshift of each object, read by
// the count kernels beside its sorted coordinates.
#include <math.h>

#include "cute_internal.h"
#include "runtime.h"

using namespace cute;

namespace {

// out[i] = in[index of sorted point i]; bad: a non-finite value
__global__ __launch_bounds__(256) void k_gather_values(const P64* __restrict__ p64, int64_t n,
                                                       const double* __restrict__ in,
                                                       double* __restrict__ out,
                                                       uint32_t* __restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i >= n) return;
    const double v = in[p64[i].idx];
    if (!isfinite(v)) atomicOr(bad, 1u);
    out[i] = v;
}

}  // namespace

namespace cute {

cute_status gather_values(const GridHost& g, const double* in, bool on_device, double* out,
                          hipStream_t s) {
    if (g.n == 0) return CUTE_OK;
    TempList tmp(s);
    const double* src = in;
    if (!on_device) {
        double* d = nullptr;
        cute_status st = tmp.alloc(&d, (size_t)g.n);
        if (st != CUTE_OK) return st;
        CUTE_HIP(hipMemcpyAsync(d, in, (size_t)g.n * sizeof(double), hipMemcpyHostToDevice, s));
        src = d;
    }
    uint32_t* bad = nullptr;
    cute_status st = tmp.alloc(&bad, 1);
    if (st != CUTE_OK) return st;
    CUTE_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_gather_values, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g.p64,
                       g.n, src, out, bad);
    CUTE_HIP(hipGetLastError());
    uint32_t hbad = 0;
    CUTE_HIP(hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CUTE_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(CUTE_E_INVALID_ARG, "non-finite redshift");
    return CUTE_OK;
}

}  // namespace cute
