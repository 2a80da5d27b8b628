// Owned device allocations and HIP error checks shared by the host-side
// sources of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mxp_internal.h"

namespace mxp {

#define HIP_CHECK(expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) fail(MXP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Owned device allocation.
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t want) {
        if (want <= bytes) return;
        release();
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(MXP_ERR_OOM, "device allocation of " + std::to_string(want) + " bytes failed");
        }
        bytes = want;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

}  // namespace mxp
