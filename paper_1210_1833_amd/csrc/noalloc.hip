// The pair count without allocation: every device temporary of the call
// lives in one fixed array per GPU (the entry point for callers that cannot
// allocate device memory). Host side plus the array itself.
#include <mutex>
#include <string>

#include "cute_internal.h"
#include "runtime.h"

namespace {

constexpr size_t kScratchBytes = (size_t)CUTE_NOALLOC_SCRATCH_BYTES;

// Each GPU the library runs on holds its own copy of this array until the
// process ends. In host code the name is only a stand-in for the symbol: the
// device address comes from hipGetSymbolAddress, once per device, and only
// that address is ever handed to kernels or copies.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    bool ready = false;
    unsigned char* ptr = nullptr;   // device address of this GPU's scratch
    hipEvent_t events[2] = {nullptr, nullptr};
};

constexpr int kMaxDevices = 64;
std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// First call on a device (which is current): look up the array's address and
// make the two timing events the counts reuse.
cute_status device_scratch(int dev, const DeviceScratch** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceScratch& d = g_dev[dev];
    if (!d.ready) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return cute::hip_status(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr) return cute::fail(CUTE_E_DEVICE, "scratch symbol has no device address");
        for (int k = 0; k < 2; k++) {
            e = hipEventCreate(&d.events[k]);
            if (e != hipSuccess) {
                if (k == 1) (void)hipEventDestroy(d.events[0]);
                d.events[0] = d.events[1] = nullptr;
                return cute::hip_status(e, "hipEventCreate");
            }
        }
        d.ptr = static_cast<unsigned char*>(p);
        d.ready = true;
    }
    *out = &d;
    return CUTE_OK;
}

}  // namespace

extern "C" cute_status cute_count_pairs_noalloc(const cute_grid* a, const cute_grid* b,
                                                const cute_binning* bins, cute_precision prec,
                                                uint64_t* counts, int32_t counts_on_device,
                                                cute_count_stats* st, void* stream) {
    int dev = 0;
    cute_status s = cute::ensure_device_ready(&dev);
    if (s != CUTE_OK) return s;
    if (dev < 0 || dev >= kMaxDevices)
        return cute::fail(CUTE_E_UNSUPPORTED, "device index beyond " + std::to_string(kMaxDevices));
    const DeviceScratch* d = nullptr;
    if ((s = device_scratch(dev, &d)) != CUTE_OK) return s;
    cute::FixedArea fa;
    fa.base = d->ptr;
    fa.cap = kScratchBytes;
    fa.events[0] = d->events[0];
    fa.events[1] = d->events[1];
    return cute::count_pairs_fixed(a, b, bins, prec, counts, counts_on_device, st, stream, &fa);
}
