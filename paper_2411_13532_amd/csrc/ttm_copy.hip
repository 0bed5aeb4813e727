// ttm_copy.hip -- a plain device copy used as the practical HBM ceiling (the
// role a STREAM copy plays in the paper's Sec. 5.1 measurements) and as the
// known-size reference for hardware byte counters.
//
// Each workgroup moves blocks of COPY_U x 256 16-byte words: every lane first
// issues its COPY_U loads (word tid, tid + 256, ...), all independent and in
// flight together, then its COPY_U stores, so a wave keeps 16 KiB of reads
// outstanding instead of one 1 KiB load per loop trip.
#include <algorithm>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

constexpr int COPY_U = 8;
constexpr int COPY_THREADS = 256;
constexpr int64_t COPY_BLOCK = int64_t(COPY_U) * COPY_THREADS;   // 16-byte words per block trip

__global__ void __launch_bounds__(COPY_THREADS) k_stream_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                              int64_t n16) {
    const int tid = threadIdx.x;
    const int64_t step = int64_t(gridDim.x) * COPY_BLOCK;
    for (int64_t b = int64_t(blockIdx.x) * COPY_BLOCK; b < n16; b += step) {
        u32x4 v[COPY_U];
        if (b + COPY_BLOCK <= n16) {
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) v[u] = __builtin_nontemporal_load(src + b + u * COPY_THREADS + tid);
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) __builtin_nontemporal_store(v[u], dst + b + u * COPY_THREADS + tid);
        } else {
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) {
                const int64_t i = b + u * COPY_THREADS + tid;
                if (i < n16) v[u] = src[i];
            }
#pragma unroll
            for (int u = 0; u < COPY_U; ++u) {
                const int64_t i = b + u * COPY_THREADS + tid;
                if (i < n16) dst[i] = v[u];
            }
        }
    }
}

}  // namespace ttm

extern "C" int ttm_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
    using namespace ttm;
    if (!dst || !src || bytes == 0 || bytes % 16 != 0 || !aligned(dst, 16) || !aligned(src, 16))
        return TTM_ERR_INVALID_ARG;
    if (overlaps(dst, bytes, src, bytes)) return TTM_ERR_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n16 = int64_t(bytes / 16);
    // eight workgroups per compute unit at a time, each looping over blocks
    const int64_t blocks = std::min<int64_t>(ceil_div(n16, COPY_BLOCK), int64_t(device_cu_count()) * 8);
    return launch("ttm_stream_copy", st, [&] {
        hipLaunchKernelGGL(k_stream_copy, dim3(unsigned(blocks)), dim3(COPY_THREADS), 0, st, static_cast<u32x4 *>(dst),
                           static_cast<const u32x4 *>(src), n16);
    });
}
