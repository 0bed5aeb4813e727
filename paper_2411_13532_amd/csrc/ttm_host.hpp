// ttm_host.hpp -- host-side helpers shared by the libttm translation units:
// argument checks, launch bracketing for per-kernel timing, status codes.
#pragma once
#include <hip/hip_runtime.h>
#include <atomic>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ttm.h"

namespace ttm {

// True when [a, a+na) and [b, b+nb) (bytes) overlap.
inline bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline size_t dtype_size(int dt) {
    switch (dt) {
        case TTM_F64: return 8;
        case TTM_F32: return 4;
        case TTM_BF16: return 2;
        default: return 0;
    }
}

// Product of positive sizes with an overflow guard (returns -1 on overflow).
inline int64_t checked_prod(int64_t a, int64_t b) {
    if (a <= 0 || b <= 0) return -1;
    if (a > (int64_t(1) << 62) / b) return -1;
    return a * b;
}

// Per-kernel timing (see ttm_timing_enable).  Every launch goes through
// launch_begin / launch_end, which record HIP events when timing is on.
bool timing_on();
void launch_begin(const char *name, hipStream_t s);
void launch_end(hipStream_t s);

// Runs one kernel launch expression, bracketing it for timing, and maps a
// launch failure to TTM_ERR_HIP.
template <typename F>
inline int launch(const char *name, hipStream_t s, F &&f) {
    launch_begin(name, s);
    f();
    hipError_t e = hipGetLastError();
    launch_end(s);
    return e == hipSuccess ? TTM_OK : TTM_ERR_HIP;
}

// Raises the dynamic LDS limit of one kernel for the current device, once per
// device and process: `done` holds one bit per device id.  Concurrent first
// calls only set the same attribute twice; a device's bit is published after
// its call succeeded.
inline int ensure_lds_limit(const void *kern, size_t lds, std::atomic<uint64_t> &done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TTM_ERR_HIP;
    const uint64_t bit = dev >= 0 && dev < 64 ? uint64_t(1) << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return TTM_OK;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
        return TTM_ERR_HIP;
    done.fetch_or(bit, std::memory_order_release);
    return TTM_OK;
}

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Slab-kernel selection set by ttm_set_slab_kernel (0 automatic, 1 register-staged,
// 2 direct-to-LDS 256-byte chunks, 3 X and C through LDS for bf16 X).
int slab_kernel_mode();

}  // namespace ttm
