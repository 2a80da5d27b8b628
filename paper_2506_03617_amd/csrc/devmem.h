// Owned device allocations, the allocator they come from, and HIP error
// checks shared by the host-side sources of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <string>

#include "mxp_internal.h"

namespace mxp {

#define HIP_CHECK(expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) fail(MXP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Counts of one context's device allocations (shared with its problems and
// networks).  `late` counts allocations made after a call had reserved its
// workspace, i.e. in the middle of its work.
struct AllocStats {
    std::atomic<int64_t> allocs{0}, frees{0}, live{0}, peak{0}, late{0};
};

// Where device memory comes from: the caller's hooks, or hipMalloc / hipFree
// when the context was created without them.
struct Allocator {
    mxp_alloc_fn alloc = nullptr;
    mxp_free_fn release = nullptr;
    void* user = nullptr;
    std::shared_ptr<AllocStats> stats;

    void* get(size_t bytes) const {
        void* p = nullptr;
        if (alloc) {
            p = alloc(bytes, user);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p && stats) {
            stats->allocs++;
            const int64_t now = stats->live += int64_t(bytes);
            int64_t pk = stats->peak.load();
            while (now > pk && !stats->peak.compare_exchange_weak(pk, now)) {
            }
        }
        return p;
    }
    void put(void* p, size_t bytes) const {
        if (!p) return;
        if (release) release(p, user);
        else (void)hipFree(p);
        if (stats) {
            stats->frees++;
            stats->live -= int64_t(bytes);
        }
    }
};

// The allocator of the entry point running on this thread, and whether that
// call has already reserved its workspace (defined in api.cpp).
extern thread_local const Allocator* t_alloc;
extern thread_local bool t_reserved;

struct AllocScope {
    const Allocator* prev;
    bool prev_reserved;
    explicit AllocScope(const Allocator& a) : prev(t_alloc), prev_reserved(t_reserved) {
        t_alloc = &a;
        t_reserved = false;
    }
    ~AllocScope() {
        t_alloc = prev;
        t_reserved = prev_reserved;
    }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

// Owned device allocation from the allocator of the entry point that made it.
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    Allocator from;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        from.put(p, bytes);
        p = nullptr;
        bytes = 0;
    }
    // Grows to at least `want` bytes (contents are not kept).  Every call of
    // the library returns only after its device work has completed, so an
    // old buffer is idle when it is replaced.
    void ensure(size_t want) {
        if (want <= bytes) return;
        if (!t_alloc) fail(MXP_ERR_HIP, "internal: device allocation outside an entry point");
        release();
        if (t_reserved && t_alloc->stats) t_alloc->stats->late++;
        p = t_alloc->get(want);
        if (!p) fail(MXP_ERR_OOM, "device allocation of " + std::to_string(want) + " bytes failed");
        from = *t_alloc;
        bytes = want;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

}  // namespace mxp
