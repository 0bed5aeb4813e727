// ttm_reorder.hip -- moving a 3-way field between directional layouts, and
// accumulating into another layout (Sec. 4.1: every direction has its own
// layout, in which that direction's lines are contiguous; Sec. 5.3 counts
// these reorders in the data movement of the transport equation).
//
// Y's axis k is X's axis perm[k].  Two kernels:
//  * the contiguous axis stays (perm[2] == 2): whole rows move, each
//    workgroup copying a 4 KiB piece of a row with 16-byte accesses;
//  * the contiguous axis changes: 64 x 64 tiles of the plane (X's axis q that
//    becomes Y's contiguous axis) x (X's contiguous axis), one tile per
//    workgroup and index of the third axis, staged through LDS: read along
//    X's rows, written along Y's rows, both with 16-byte accesses where the
//    rows allow it (odd LDS row stride: the column reads of the write phase
//    hit distinct banks).
// Accumulation reads Y, adds in the element type and writes it back.
#include <algorithm>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

constexpr int RO_TILE = 64;
constexpr int RO_THREADS = 256;

struct ReorderArgs {
    const void *X;
    void *Y;
    int64_t n[3];        // X dims
    int64_t ys[3];       // Y stride (elements) of each X axis
    int q;               // X axis that is contiguous in Y
    int o;               // the remaining axis (neither q nor 2)
    int64_t tiles2, tilesq;
    int vec;             // 16-byte accesses: n[2] and n[q] are multiples of the vector width, pointers aligned
};

template <typename T, bool ACC>
__device__ __forceinline__ void put(T *y, T v) {
    if constexpr (ACC) *y = *y + v;
    else *y = v;
}

// Contiguous axis unchanged: rows of n[2] elements move as blocks.  Row
// (i0, i1) of X goes to offset i0 * ys[0] + i1 * ys[1] of Y.  blockIdx.x:
// 4 KiB piece of the row, blockIdx.y: row (continued in z).  (Eight rows
// per workgroup with all their loads in flight measured slower: 3.6 against
// 5.3 TB/s on 512^3 float64.)
template <typename T, bool ACC>
__global__ void __launch_bounds__(RO_THREADS) k_reorder_rows(const ReorderArgs a) {
    constexpr int V = 16 / sizeof(T);
    const int64_t row = int64_t(blockIdx.z) * gridDim.y + blockIdx.y;
    if (row >= a.n[0] * a.n[1]) return;
    const int64_t i0 = row / a.n[1], i1 = row - i0 * a.n[1];
    const T *xr = static_cast<const T *>(a.X) + row * a.n[2];
    T *yr = static_cast<T *>(a.Y) + i0 * a.ys[0] + i1 * a.ys[1];
    const int64_t e0 = int64_t(blockIdx.x) * RO_THREADS * V;
    if (a.vec) {
        typedef T TV __attribute__((ext_vector_type(V)));
        const int64_t e = e0 + int64_t(threadIdx.x) * V;
        if (e < a.n[2]) {
            const TV v = *reinterpret_cast<const TV *>(xr + e);
            TV *d = reinterpret_cast<TV *>(yr + e);
            if constexpr (ACC) *d = *d + v;
            else *d = v;
        }
    } else {
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int64_t e = e0 + int64_t(u) * RO_THREADS + threadIdx.x;
            if (e < a.n[2]) put<T, ACC>(yr + e, xr[e]);
        }
    }
}

// Contiguous axis changes: tile (t2, tq) of the (i_q, i_2) plane at index i_o
// of the third axis.  X element (i_o, i_q, i_2) is read along i_2 and written
// to Y at i_o * ys[o] + i_2 * ys[2] + i_q, along i_q.
template <typename T, bool ACC>
__global__ void __launch_bounds__(RO_THREADS) k_reorder_tiles(const ReorderArgs a) {
    constexpr int V = 16 / sizeof(T);
    constexpr int LD = RO_TILE + 1;                   // odd row stride (elements)
    __shared__ T tile[RO_TILE * LD];                  // tile[iq_local * LD + i2_local]
    const int64_t b = blockIdx.x;
    const int64_t per_o = a.tiles2 * a.tilesq;
    const int64_t io = b / per_o;
    const int64_t rem = b - io * per_o;
    const int64_t tq = rem / a.tiles2, t2 = rem - tq * a.tiles2;
    const int64_t q0 = tq * RO_TILE, c0 = t2 * RO_TILE;
    const int64_t nq = a.n[a.q], n2 = a.n[2];
    const int64_t sxq = a.q == 0 ? a.n[1] * a.n[2] : a.n[2];
    const int64_t sxo = a.o == 0 ? a.n[1] * a.n[2] : a.n[2];
    const T *xb = static_cast<const T *>(a.X) + io * sxo + q0 * sxq + c0;
    T *yb = static_cast<T *>(a.Y) + io * a.ys[a.o] + c0 * a.ys[2] + q0;
    const int tid = threadIdx.x;
    const bool full = q0 + RO_TILE <= nq && c0 + RO_TILE <= n2;

    // read: rows of X (fixed i_q) along i_2
    if (a.vec && full) {
        typedef T TV __attribute__((ext_vector_type(V)));
        constexpr int VPR = RO_TILE / V;              // vectors per row
        constexpr int ROWS = RO_THREADS / VPR;        // rows per step
#pragma unroll
        for (int r0 = 0; r0 < RO_TILE; r0 += ROWS) {
            const int r = r0 + tid / VPR, c = (tid % VPR) * V;
            const TV v = *reinterpret_cast<const TV *>(xb + r * sxq + c);
#pragma unroll
            for (int k = 0; k < V; ++k) tile[r * LD + c + k] = v[k];
        }
    } else {
        for (int idx = tid; idx < RO_TILE * RO_TILE; idx += RO_THREADS) {
            const int r = idx / RO_TILE, c = idx % RO_TILE;
            if (q0 + r < nq && c0 + c < n2) tile[r * LD + c] = xb[r * sxq + c];
        }
    }
    __syncthreads();
    // write: rows of Y (fixed i_2) along i_q
    if (a.vec && full) {
        typedef T TV __attribute__((ext_vector_type(V)));
        constexpr int VPR = RO_TILE / V;
        constexpr int ROWS = RO_THREADS / VPR;
#pragma unroll
        for (int c0l = 0; c0l < RO_TILE; c0l += ROWS) {
            const int c = c0l + tid / VPR, r = (tid % VPR) * V;
            TV v;
#pragma unroll
            for (int k = 0; k < V; ++k) v[k] = tile[(r + k) * LD + c];
            TV *d = reinterpret_cast<TV *>(yb + c * a.ys[2] + r);
            if constexpr (ACC) *d = *d + v;
            else *d = v;
        }
    } else {
        for (int idx = tid; idx < RO_TILE * RO_TILE; idx += RO_THREADS) {
            const int c = idx / RO_TILE, r = idx % RO_TILE;
            if (q0 + r < nq && c0 + c < n2) put<T, ACC>(yb + c * a.ys[2] + r, tile[r * LD + c]);
        }
    }
}

template <typename T>
static int launch_reorder(const ReorderArgs &a, bool rows, int acc, hipStream_t st) {
    constexpr int V = 16 / sizeof(T);
    if (rows) {
        const int64_t nrows = a.n[0] * a.n[1];
        const int64_t gy = std::min<int64_t>(nrows, 65535), gz = ceil_div(nrows, gy);
        dim3 grid(unsigned(ceil_div(a.n[2], int64_t(RO_THREADS) * V)), unsigned(gy), unsigned(gz));
        return launch("ttm_reorder", st, [&] {
            if (acc) hipLaunchKernelGGL((k_reorder_rows<T, true>), grid, dim3(RO_THREADS), 0, st, a);
            else hipLaunchKernelGGL((k_reorder_rows<T, false>), grid, dim3(RO_THREADS), 0, st, a);
        });
    }
    const int64_t ntiles = a.tiles2 * a.tilesq * a.n[a.o];
    return launch("ttm_reorder", st, [&] {
        if (acc) hipLaunchKernelGGL((k_reorder_tiles<T, true>), dim3(unsigned(ntiles)), dim3(RO_THREADS), 0, st, a);
        else hipLaunchKernelGGL((k_reorder_tiles<T, false>), dim3(unsigned(ntiles)), dim3(RO_THREADS), 0, st, a);
    });
}

}  // namespace ttm

extern "C" int ttm_reorder(const int64_t *dims, const int *perm, const void *X, void *Y, int dtype, int accumulate,
                           void *stream) {
    using namespace ttm;
    if (!dims || !perm || !X || !Y) return TTM_ERR_INVALID_ARG;
    if (dtype != TTM_F32 && dtype != TTM_F64) return TTM_ERR_UNSUPPORTED;
    int seen[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        if (perm[k] < 0 || perm[k] > 2 || seen[perm[k]]) return TTM_ERR_INVALID_ARG;
        seen[perm[k]] = 1;
    }
    for (int k = 0; k < 3; ++k)
        if (dims[k] < 1 || dims[k] > (int64_t(1) << 31)) return TTM_ERR_INVALID_ARG;
    const int64_t total = checked_prod(checked_prod(dims[0], dims[1]), dims[2]);
    if (total < 0) return TTM_ERR_INVALID_ARG;
    const size_t es = dtype_size(dtype);
    if (!aligned(X, es) || !aligned(Y, es)) return TTM_ERR_INVALID_ARG;
    if (overlaps(X, size_t(total) * es, Y, size_t(total) * es)) return TTM_ERR_ALIAS;
    ReorderArgs a;
    a.X = X;
    a.Y = Y;
    for (int k = 0; k < 3; ++k) a.n[k] = dims[k];
    const int64_t yd[3] = {dims[perm[0]], dims[perm[1]], dims[perm[2]]};
    const int64_t sy[3] = {yd[1] * yd[2], yd[2], 1};
    for (int k = 0; k < 3; ++k) a.ys[perm[k]] = sy[k];
    const int V = int(16 / es);
    const bool rows = perm[2] == 2;
    a.q = perm[2];
    a.o = 3 - a.q - 2;            // the axis that is neither q nor 2 (q != 2 here)
    if (rows) a.o = 0;
    a.tiles2 = ceil_div(dims[2], RO_TILE);
    a.tilesq = rows ? 1 : ceil_div(dims[a.q], RO_TILE);
    a.vec = aligned(X, 16) && aligned(Y, 16) && dims[2] % V == 0 && (rows || dims[a.q] % V == 0);
    if (!rows && a.tiles2 * a.tilesq * dims[a.o] > 0x7fffffffLL) return TTM_ERR_UNSUPPORTED;
    if (rows && ceil_div(dims[0] * dims[1], 65535) > 65535) return TTM_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return dtype == TTM_F64 ? launch_reorder<double>(a, rows, accumulate, st)
                            : launch_reorder<float>(a, rows, accumulate, st);
}
