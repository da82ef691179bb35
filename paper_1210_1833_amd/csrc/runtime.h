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

// Set up the library's memory pool on the current device (once per device).
cute_status ensure_device_ready(int* device);

// Stream-ordered device allocation from the library's own pool (its freed
// blocks are kept for reuse up to a bound, without changing the device's
// default pool for the rest of the process). Every device allocation of the
// library goes through here, so that a test can make the n-th one fail: while
// the environment sets CUTE_TEST_FAIL_ALLOC=n (n > 0), every n-th call
// reports CUTE_E_OUT_OF_MEMORY instead of allocating.
cute_status dev_malloc_async(void** p, size_t bytes, hipStream_t s);
bool inject_alloc_failure();

template <typename T>
cute_status dalloc(T** p, size_t count, hipStream_t s) {
    *p = nullptr;
    if (count == 0) count = 1;
    return dev_malloc_async(reinterpret_cast<void**>(p), count * sizeof(T), s);
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

// Device memory for the temporaries of one call. By default each piece is a
// stream-ordered pool allocation, freed (in stream order) with the arena.
// Given a fixed area, the pieces are consecutive 256-byte-aligned slices of
// it and nothing is allocated or freed; a request beyond the area fails.
class DevArena {
  public:
    explicit DevArena(hipStream_t s) : s_(s) {}
    DevArena(hipStream_t s, unsigned char* base, size_t cap) : s_(s), base_(base), cap_(cap) {}
    bool fixed() const { return base_ != nullptr; }
    size_t capacity() const { return cap_; }
    // bytes a fixed area spends on `count` elements of T (with alignment)
    template <typename T>
    static size_t cost(size_t count) {
        return ((count ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
    }
    template <typename T>
    cute_status get(T** p, size_t count) {
        *p = nullptr;
        if (!fixed()) {
            cute_status st = dalloc(p, count, s_);
            if (st == CUTE_OK) owned_.push_back(*p);
            return st;
        }
        const size_t need = cost<T>(count);
        if (need > cap_ - used_) return scratch_full(need);
        *p = reinterpret_cast<T*>(base_ + used_);
        used_ += need;
        return CUTE_OK;
    }
    ~DevArena() {
        for (void* q : owned_) dfree(q, s_);
    }
    DevArena(const DevArena&) = delete;
    DevArena& operator=(const DevArena&) = delete;

  private:
    cute_status scratch_full(size_t need) const;
    hipStream_t s_;
    unsigned char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    std::vector<void*> owned_;
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
    bool own = true;
    explicit EventTimer(hipStream_t st) : s(st) {
        if (hipEventCreate(&a) != hipSuccess) a = nullptr;
        if (hipEventCreate(&b) != hipSuccess) b = nullptr;
        if (a) (void)hipEventRecord(a, s);
    }
    // borrowed: two events made beforehand and kept by the caller (none
    // created here); nullptr: two new events, as above
    EventTimer(hipStream_t st, const hipEvent_t* borrowed) : s(st) {
        if (borrowed) {
            a = borrowed[0];
            b = borrowed[1];
            own = false;
        } else {
            if (hipEventCreate(&a) != hipSuccess) a = nullptr;
            if (hipEventCreate(&b) != hipSuccess) b = nullptr;
        }
        if (a) (void)hipEventRecord(a, s);
    }
    EventTimer(const EventTimer&) = delete;
    EventTimer& operator=(const EventTimer&) = delete;
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
        if (!own) return;
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace cute
