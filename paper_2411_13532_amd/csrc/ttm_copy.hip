// ttm_copy.hip -- a plain device copy used as the practical HBM ceiling (the
// role BabelStream's copy plays in the paper's Sec. 5.1 measurements) and as
// the known-size reference for hardware byte counters.  Written here; each
// thread moves 16-byte words with a grid-stride loop.
#include <algorithm>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

__global__ void __launch_bounds__(256) k_stream_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, int64_t n16) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace ttm

extern "C" int ttm_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
    using namespace ttm;
    if (!dst || !src || bytes == 0 || bytes % 16 != 0 || !aligned(dst, 16) || !aligned(src, 16))
        return TTM_ERR_INVALID_ARG;
    if (overlaps(dst, bytes, src, bytes)) return TTM_ERR_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n16 = int64_t(bytes / 16);
    const int64_t blocks = std::min<int64_t>(ceil_div(n16, 256), int64_t(device_cu_count()) * 16);
    return launch("ttm_stream_copy", st, [&] {
        hipLaunchKernelGGL(k_stream_copy, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<u32x4 *>(dst),
                           static_cast<const u32x4 *>(src), n16);
    });
}
