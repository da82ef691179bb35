// Small host runtime helpers: HIP error mapping, stream-ordered allocation,
// event timing.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cute_internal.h"

namespace cute {

cute_status hip_status(hipError_t e, const char* what);

#define CUTE_HIP(call)                                                  \
    do {                                                                \
        hipError_t e__ = (call);                                        \
        if (e__ != hipSuccess) return ::cute::hip_status(e__, #call);   \
    } while (0)

// Make the default memory pool keep freed blocks (stream-ordered reuse).
cute_status ensure_device_ready(int* device);

template <typename T>
cute_status dalloc(T** p, size_t count, hipStream_t s) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), count * sizeof(T), s);
    if (e != hipSuccess) return hip_status(e, "hipMallocAsync");
    return CUTE_OK;
}

inline void dfree(void* p, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
}

// RAII list of stream-ordered temporaries.
struct TempList {
    hipStream_t s;
    std::vector<void*> ptrs;
    explicit TempList(hipStream_t st) : s(st) {}
    template <typename T>
    cute_status alloc(T** p, size_t count) {
        cute_status st = dalloc(p, count, s);
        if (st == CUTE_OK) ptrs.push_back(*p);
        return st;
    }
    ~TempList() {
        for (void* p : ptrs) dfree(p, s);
    }
};

// Pinned host memory for the small copies of one call, leased from a pool
// of buffers that are kept for reuse (never freed). The copies stay
// asynchronous: releasing the lease records an event on the call's stream,
// and the next lease of the buffer waits for it.
struct StageBuf;
class HostStage {
  public:
    explicit HostStage(hipStream_t s) : s_(s) {}
    // a buffer of at least `bytes` (contents undefined)
    cute_status get(size_t bytes, unsigned char** p);
    ~HostStage();
    HostStage(const HostStage&) = delete;
    HostStage& operator=(const HostStage&) = delete;

  private:
    hipStream_t s_;
    StageBuf* b_ = nullptr;
};

struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        if (hipEventCreate(&a) != hipSuccess) a = nullptr;
        if (hipEventCreate(&b) != hipSuccess) b = nullptr;
        if (a) (void)hipEventRecord(a, s);
    }
    // record the end (no wait)
    void stop() {
        if (a && b) (void)hipEventRecord(b, s);
    }
    // time between the two records, waiting for the end if needed
    double elapsed_ms() {
        if (!a || !b) return 0.0;
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    double stop_ms() {
        stop();
        return elapsed_ms();
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace cute
