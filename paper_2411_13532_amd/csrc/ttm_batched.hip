// ttm_batched.hip -- many small independent chains Y_k = X_k x1 A_k x2 B_k x3 C_k
// (ragged sizes, every mode at most 16) in one persistent launch.
//
// One wavefront owns one cuboid at a time, as the paper groups independent
// lines onto the lanes of one execution unit (Sec. 4.1, the SZ-grouped
// layout).  In float each mode product is a row of 16 x 16 x 4 matrix-core
// tiles (mode 3: rows (i1, i2) x columns j3; mode 2: one j2 x j3 tile per i1;
// mode 1: rows j1 x columns (j2, j3)), operands read from LDS one element per
// lane.  In double a lane keeps one input fiber in registers and produces the
// whole output fiber, reading the factor rows from LDS 16 bytes at a time at
// the same address on every lane (a broadcast).
// The inputs of a cuboid (its three factors and X, one lane-strided
// sequence) are loaded into registers while the wave still works on the
// previous cuboid, so the HBM latency of one cuboid overlaps the arithmetic of
// the one before; they then go to LDS (factor rows zero-padded, X fibers at
// odd strides: no bank conflicts).  The intermediates of modes 3 and 2 stay in
// LDS; Y is written with coalesced stores.  Waves take cuboids from a static
// longest-first order (work ~ I1*I2*I3*J3 + ...), wave w handling positions
// w, w + W, w + 2W, ... of that order; the launch shape (threads per block,
// resident blocks per compute unit) is autotuned per workload and cached.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

constexpr int BATCH_MAXN = 16;

struct alignas(16) CuboidDesc {
    int64_t ox, oa, ob, oc, oy;   // element offsets of X_k, A_k, B_k, C_k, Y_k
    int32_t d[6];                 // I1, I2, I3, J1, J2, J3
};

struct BatchArgs {
    const CuboidDesc *desc;
    int64_t count;
    const void *X, *A, *B, *C;
    void *Y;
    int fac_elems, w_elems, xv_elems;   // per-wave LDS regions (elements)
};


// Four fiber contractions at once: s[r] = sum_{e < n} U[r][e] * x[e] for
// factor rows U[r] = urow + r * P in LDS (zero-padded to a multiple of 4) and
// x in registers (x[e] = 0 for e >= n).  Every lane reads the same address (a
// broadcast), 16 bytes at a time, and whole groups of 4 past n are skipped (n
// is wave-uniform).  Four independent sums keep four LDS reads in flight.
// Rows past the factor's last read other LDS data of the same wave; their
// sums are discarded.  Fixed order of the terms.
template <typename T>
__device__ __forceinline__ void dot_rows4(const T *urow, int P, const T (&x)[BATCH_MAXN], int n, T (&s)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s[r] = T(0);
#pragma unroll
    for (int e4 = 0; e4 < BATCH_MAXN / 4; ++e4) {
        if (4 * e4 < n) {
            T u[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) __builtin_memcpy(u[r], urow + r * P + 4 * e4, sizeof u[r]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) s[r] += u[r][i] * x[4 * e4 + i];
        }
    }
}

// X of the next cuboid is loaded into registers (BATCH_PF elements per lane,
// every load issued before any is used) while the wave works on the current
// one; a larger X loads its rest at stage 0.
constexpr int BATCH_PF = 40;

// Row r = e / len for e < 4096, len <= 16: the float quotient is at least
// 1/32 away from the next integer, far more than its rounding error.
__device__ __forceinline__ int row_of(int e, float inv_len) { return int((float(e) + 0.5f) * inv_len); }

// n (<= 256) elements of a factor (rows of len), already loaded as
// r[u] = element u * 64 + lane, into LDS rows of stride P.
template <typename T>
__device__ __forceinline__ void factor_regs_to_lds(const T (&r)[4], int n, int len, int P, T *dst, int lane) {
    const float inv = 1.0f / float(len);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = u * 64 + lane;
        const int row = row_of(e, inv);
        if (e < n) dst[row * P + (e - row * len)] = r[u];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_batched(const BatchArgs a, const T *__restrict__ X, const T *__restrict__ Ag,
                                                 const T *__restrict__ Bg, const T *__restrict__ Cg,
                                                 T *__restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int wpb = blockDim.x >> 6;
    const int per_wave = a.fac_elems + a.w_elems + a.xv_elems;
    T *fac = reinterpret_cast<T *>(smem_raw) + int64_t(wave) * per_wave;
    T *W = fac + a.fac_elems;
    T *XV = W + a.w_elems;
    const int64_t total_waves = int64_t(gridDim.x) * wpb;

    // float: the three products on the matrix cores (16x16x4 tiles, operands
    // read from LDS with out-of-range elements replaced by zeros); double: the
    // vector path
    constexpr bool MF = std::is_same<T, float>::value;
    const int r16 = lane & 15, g = lane >> 4;

    // the next cuboid's X (BATCH_PF elements per lane) and three factors (at
    // most 256 elements each, 4 per lane) are loaded into registers while the
    // wave works on the current one
    T pre[BATCH_PF], pf[3][4];
    auto prefetch = [&](const CuboidDesc &d) __attribute__((always_inline)) {
        const int nx = d.d[0] * d.d[1] * d.d[2];
        const T *xs = X + d.ox;
#pragma unroll
        for (int u = 0; u < BATCH_PF; ++u) {
            if (u * 64 < nx) {   // uniform: only the rows of 64 that X fills
                const int e = u * 64 + lane;
                pre[u] = xs[e < nx ? e : nx - 1];
            }
        }
        const T *fs[3] = {Ag + d.oa, Bg + d.ob, Cg + d.oc};
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int n = d.d[3 + f] * d.d[f];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = u * 64 + lane;
                pf[f][u] = fs[f][e < n ? e : n - 1];
            }
        }
    };

    int64_t idx = int64_t(blockIdx.x) * wpb + wave;
    if (idx < a.count) prefetch(a.desc[idx]);
    for (; idx < a.count; idx += total_waves) {
        const CuboidDesc d = a.desc[idx];
        const int I1 = d.d[0], I2 = d.d[1], I3 = d.d[2], J1 = d.d[3], J2 = d.d[4], J3 = d.d[5];
        // factor rows padded to multiples of 4 (zeros); odd strides for fibers
        const int P1 = (I1 + 3) & ~3, P2 = (I2 + 3) & ~3, P3 = (I3 + 3) & ~3;
        const int SX = I3 | 1, SW = J3 | 1;
        T *As = fac, *Bs = fac + J1 * P1, *Cs = Bs + J2 * P2;
        const int nx = I1 * I2 * I3;

        // stage 0: factors into zero-padded LDS rows, X (prefetched, plus any
        // rest) into fibers of odd stride
        if constexpr (!MF) {   // the vector path reads whole padded groups of 4
            const int nfac = J1 * P1 + J2 * P2 + J3 * P3;
            for (int e = lane; e < nfac; e += 64) fac[e] = T(0);
            wave_sync();
        }
        factor_regs_to_lds(pf[0], J1 * I1, I1, P1, As, lane);
        factor_regs_to_lds(pf[1], J2 * I2, I2, P2, Bs, lane);
        factor_regs_to_lds(pf[2], J3 * I3, I3, P3, Cs, lane);
        const float inv3 = 1.0f / float(I3);
#pragma unroll
        for (int u = 0; u < BATCH_PF; ++u) {
            if (u * 64 < nx) {
                const int e = u * 64 + lane;
                const int f = row_of(e, inv3);
                if (e < nx) XV[f * SX + (e - f * I3)] = pre[u];
            }
        }
        for (int base = BATCH_PF * 64; base < nx; base += 16 * 64) {
            T r[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = base + u * 64 + lane;
                r[u] = X[d.ox + (e < nx ? e : nx - 1)];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = base + u * 64 + lane;
                const int f = row_of(e, inv3);
                if (e < nx) XV[f * SX + (e - f * I3)] = r[u];
            }
        }
        wave_sync();
        if (idx + total_waves < a.count) prefetch(a.desc[idx + total_waves]);

        if constexpr (MF) {
            // stage 1 (mode 3): W[m][j3] = sum_i3 X[m][i3] C[j3][i3], m = (i1, i2):
            // 16-row blocks of m, k steps of 4 along i3
            {
                const int M = I1 * I2, KS = (I3 + 3) >> 2;
                float bf[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = 4 * ks + g;
                    const bool ok = ks < KS && k < I3 && r16 < J3;
                    bf[ks] = ok ? Cs[r16 * P3 + k] : 0.f;
                }
                for (int m0 = 0; m0 < M; m0 += 16) {
                    const int m = m0 + r16;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        if (ks < KS) {
                            const int k = 4 * ks + g;
                            const bool ok = m < M && k < I3;
                            acc = mfma_f32(ok ? XV[ok ? m * SX + k : 0] : 0.f, bf[ks], acc);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = m0 + 4 * g + r;
                        if (row < M && r16 < J3) W[row * SW + r16] = acc[r];
                    }
                }
            }
            wave_sync();
            // stage 2 (mode 2): V[i1][j2][j3] = sum_i2 B[j2][i2] W[i1][i2][j3], one
            // 16 x 16 tile per i1; V goes to X's region at row stride NCS
            const int NC = J2 * J3, NCS = NC | 1;
            {
                const int KS = (I2 + 3) >> 2;
                float af[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = 4 * ks + g;
                    const bool ok = ks < KS && k < I2 && r16 < J2;
                    af[ks] = ok ? Bs[r16 * P2 + k] : 0.f;
                }
                for (int i1 = 0; i1 < I1; ++i1) {
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        if (ks < KS) {
                            const int k = 4 * ks + g;
                            const bool ok = k < I2 && r16 < J3;
                            acc = mfma_f32(af[ks], ok ? W[ok ? (i1 * I2 + k) * SW + r16 : 0] : 0.f, acc);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j2 = 4 * g + r;
                        if (j2 < J2 && r16 < J3) XV[i1 * NCS + j2 * J3 + r16] = acc[r];
                    }
                }
            }
            wave_sync();
            // stage 3 (mode 1): Y[j1][c] = sum_i1 A[j1][i1] V[i1][c], c = (j2, j3):
            // 16-column blocks of c
            {
                const int KS = (I1 + 3) >> 2;
                float af[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = 4 * ks + g;
                    const bool ok = ks < KS && k < I1 && r16 < J1;
                    af[ks] = ok ? As[r16 * P1 + k] : 0.f;
                }
                for (int c0 = 0; c0 < NC; c0 += 16) {
                    const int c = c0 + r16;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        if (ks < KS) {
                            const int k = 4 * ks + g;
                            const bool ok = k < I1 && c < NC;
                            acc = mfma_f32(af[ks], ok ? XV[ok ? k * NCS + c : 0] : 0.f, acc);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j1 = 4 * g + r;
                        if (j1 < J1 && c < NC) Y[d.oy + int64_t(j1) * NC + c] = acc[r];
                    }
                }
            }
            wave_sync();
        } else {
            // stage 1 (mode 3): fiber f = (i1, i2): W[f][j3] = sum_i3 C[j3][i3] X[f][i3]
            for (int f = lane; f < I1 * I2; f += 64) {
                T x[BATCH_MAXN];
#pragma unroll
                for (int e = 0; e < BATCH_MAXN; ++e) x[e] = e < I3 ? XV[f * SX + e] : T(0);
                for (int j = 0; j < J3; j += 4) {
                    T o[4];
                    dot_rows4(Cs + j * P3, P3, x, I3, o);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j + r < J3) W[f * SW + j + r] = o[r];
                }
            }
            wave_sync();

            // stage 2 (mode 2): fiber (i1, j3) along i2: V[i1][j2][j3] = sum_i2 B[j2][i2] W[i1][i2][j3]
            // V overwrites X's region (X is no longer needed)
            for (int it = lane; it < I1 * J3; it += 64) {
                const int i1 = it / J3, j3 = it - i1 * J3;
                T w[BATCH_MAXN];
#pragma unroll
                for (int e = 0; e < BATCH_MAXN; ++e) w[e] = e < I2 ? W[(i1 * I2 + e) * SW + j3] : T(0);
                for (int j = 0; j < J2; j += 4) {
                    T o[4];
                    dot_rows4(Bs + j * P2, P2, w, I2, o);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j + r < J2) XV[(i1 * J2 + j + r) * J3 + j3] = o[r];
                }
            }
            wave_sync();

            // stage 3 (mode 1): fiber (j2, j3) along i1: Y[j1][j2][j3] = sum_i1 A[j1][i1] V[i1][j2][j3]
            const int n23 = J2 * J3;
            for (int it = lane; it < n23; it += 64) {
                T v[BATCH_MAXN];
#pragma unroll
                for (int e = 0; e < BATCH_MAXN; ++e) v[e] = e < I1 ? XV[e * n23 + it] : T(0);
                for (int j = 0; j < J1; j += 4) {
                    T o[4];
                    dot_rows4(As + j * P1, P1, v, I1, o);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j + r < J1) Y[d.oy + int64_t(j + r) * n23 + it] = o[r];
                }
            }
            wave_sync();
        }
    }
}

}  // namespace ttm

using namespace ttm;

struct ttm_batched_plan {
    int64_t count = 0;
    int dtype = TTM_F32;
    int device = 0;
    size_t esz = 4;
    std::vector<int64_t> dims;
    int64_t totals[5] = {0, 0, 0, 0, 0};
    CuboidDesc *d_desc = nullptr;
    int fac_elems = 0, w_elems = 0, xv_elems = 0;
    int threads = 256, blocks_per_cu = 2;
    int cu_count = 256;
    std::string tune_cache, tune_key;
    // graph replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    BatchArgs graph_args;
    const void *graph_ptrs[5];
    void *graph_params[6];
};

namespace {

size_t lds_per_wave(const ttm_batched_plan *p) { return size_t(p->fac_elems + p->w_elems + p->xv_elems) * p->esz; }

int max_blocks_per_cu(const ttm_batched_plan *p, int threads) {
    const size_t per_block = lds_per_wave(p) * size_t(threads / 64);
    const size_t lds_cu = 160 * 1024;
    int b = int(lds_cu / std::max<size_t>(per_block, 1));
    const int waves_cap = 32 / (threads / 64);   // resident waves per compute unit
    return std::max(0, std::min(b, waves_cap));
}

BatchArgs make_args(const ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y) {
    BatchArgs a;
    a.desc = p->d_desc;
    a.count = p->count;
    a.X = X; a.A = A; a.B = B; a.C = C; a.Y = Y;
    a.fac_elems = p->fac_elems;
    a.w_elems = p->w_elems;
    a.xv_elems = p->xv_elems;
    return a;
}

const void *kernel_ptr(int dtype) {
    return dtype == TTM_F64 ? reinterpret_cast<const void *>(&k_batched<double>)
                            : reinterpret_cast<const void *>(&k_batched<float>);
}

int launch_batched(const ttm_batched_plan *p, const BatchArgs &a, int threads, int bpc, hipStream_t st,
                   int64_t nblocks_override = 0) {
    const size_t lds = lds_per_wave(p) * size_t(threads / 64);
    int64_t nblocks = nblocks_override ? nblocks_override : int64_t(p->cu_count) * bpc;
    const int64_t useful = ceil_div(p->count, threads / 64);
    if (nblocks > useful) nblocks = useful;
    if (nblocks < 1) nblocks = 1;
    return launch("ttm_batched", st, [&] {
        if (p->dtype == TTM_F64)
            hipLaunchKernelGGL(k_batched<double>, dim3(unsigned(nblocks)), dim3(threads), lds, st, a,
                               static_cast<const double *>(a.X), static_cast<const double *>(a.A),
                               static_cast<const double *>(a.B), static_cast<const double *>(a.C),
                               static_cast<double *>(a.Y));
        else
            hipLaunchKernelGGL(k_batched<float>, dim3(unsigned(nblocks)), dim3(threads), lds, st, a,
                               static_cast<const float *>(a.X), static_cast<const float *>(a.A),
                               static_cast<const float *>(a.B), static_cast<const float *>(a.C),
                               static_cast<float *>(a.Y));
    });
}

int check_buffers(const ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C,
                  const void *Y) {
    if (!p || !X || !A || !B || !C || !Y) return TTM_ERR_INVALID_ARG;
    const size_t e = p->esz;
    if (!aligned(X, e) || !aligned(A, e) || !aligned(B, e) || !aligned(C, e) || !aligned(Y, e))
        return TTM_ERR_INVALID_ARG;
    const size_t ny = size_t(p->totals[4]) * e;
    if (overlaps(Y, ny, X, size_t(p->totals[0]) * e) || overlaps(Y, ny, A, size_t(p->totals[1]) * e) ||
        overlaps(Y, ny, B, size_t(p->totals[2]) * e) || overlaps(Y, ny, C, size_t(p->totals[3]) * e))
        return TTM_ERR_ALIAS;
    return TTM_OK;
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

// Cache entries are one JSON object per line inside a JSON object:
//   {
//   "<key>": {"threads": T, "blocks_per_cu": B, "ms": M},
//   ...
//   }
bool cache_lookup(const std::string &path, const std::string &key, int &threads, int &bpc) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string needle = "\"" + key + "\":";
    while (fgets(line, sizeof line, f)) {
        if (strstr(line, needle.c_str()) != line) continue;
        const char *t = strstr(line, "\"threads\":");
        const char *b = strstr(line, "\"blocks_per_cu\":");
        if (t && b) {
            threads = atoi(t + 10);
            bpc = atoi(b + 16);
            found = threads == 64 || threads == 128 || threads == 256;
        }
        break;
    }
    fclose(f);
    return found && bpc >= 1;
}

bool cache_store(const std::string &path, const std::string &key, int threads, int bpc, double ms) {
    std::vector<std::string> keep;
    if (FILE *f = fopen(path.c_str(), "r")) {
        char line[1024];
        const std::string needle = "\"" + key + "\":";
        while (fgets(line, sizeof line, f)) {
            if (line[0] != '"') continue;
            if (strstr(line, needle.c_str()) == line) continue;
            std::string s(line);
            while (!s.empty() && (s.back() == '\n' || s.back() == ',' || s.back() == ' ')) s.pop_back();
            keep.push_back(s);
        }
        fclose(f);
    }
    char buf[512];
    snprintf(buf, sizeof buf, "\"%s\": {\"threads\": %d, \"blocks_per_cu\": %d, \"ms\": %.6f}", key.c_str(), threads,
             bpc, ms);
    keep.push_back(buf);
    const std::string tmp = path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    for (size_t i = 0; i < keep.size(); ++i) fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    return rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

extern "C" {

int ttm_batched_plan_create(int64_t count, const int64_t *dims_host, int dtype, int math, const char *tune_cache,
                            void *stream, ttm_batched_plan **out) {
    if (!out) return TTM_ERR_INVALID_ARG;
    *out = nullptr;
    if (count < 1 || !dims_host) return TTM_ERR_INVALID_ARG;
    if (!((dtype == TTM_F32 && math == TTM_MATH_F32) || (dtype == TTM_F64 && math == TTM_MATH_F64)))
        return TTM_ERR_UNSUPPORTED;
    if (count > (int64_t(1) << 31)) return TTM_ERR_UNSUPPORTED;
    for (int64_t k = 0; k < count * 6; ++k)
        if (dims_host[k] < 1 || dims_host[k] > BATCH_MAXN) return TTM_ERR_INVALID_ARG;

    ttm_batched_plan *p = new ttm_batched_plan();
    p->count = count;
    p->dtype = dtype;
    p->esz = dtype == TTM_F64 ? 8 : 4;
    p->dims.assign(dims_host, dims_host + count * 6);

    // offsets in input order, then the longest-first processing order
    std::vector<CuboidDesc> desc(static_cast<size_t>(count));
    std::vector<int64_t> work(static_cast<size_t>(count));
    int64_t o[5] = {0, 0, 0, 0, 0};
    for (int64_t k = 0; k < count; ++k) {
        const int64_t *d = dims_host + 6 * k;
        CuboidDesc &c = desc[size_t(k)];
        c.ox = o[0]; c.oa = o[1]; c.ob = o[2]; c.oc = o[3]; c.oy = o[4];
        for (int n = 0; n < 6; ++n) c.d[n] = int32_t(d[n]);
        o[0] += d[0] * d[1] * d[2];
        o[1] += d[3] * d[0];
        o[2] += d[4] * d[1];
        o[3] += d[5] * d[2];
        o[4] += d[3] * d[4] * d[5];
        work[size_t(k)] = d[0] * d[1] * d[2] * d[5] + d[0] * d[1] * d[4] * d[5] + d[0] * d[3] * d[4] * d[5];
        p->fac_elems = std::max<int>(p->fac_elems, int(d[3] * round_up(d[0], 4) + d[4] * round_up(d[1], 4) +
                                                       d[5] * round_up(d[2], 4)));
        p->w_elems = std::max<int>(p->w_elems, int(d[0] * d[1] * (d[5] | 1)));
        p->xv_elems = std::max<int>(p->xv_elems, int(std::max(d[0] * d[1] * (d[2] | 1), d[0] * ((d[4] * d[5]) | 1))));
    }
    for (int n = 0; n < 5; ++n) p->totals[n] = o[n];
    // dot_rows4 reads up to three rows (of at most 16) past a factor's last
    p->fac_elems += 3 * BATCH_MAXN;
    // keep every region 16-byte aligned
    const int al = int(16 / p->esz);
    p->fac_elems = int(round_up(p->fac_elems, al));
    p->w_elems = int(round_up(p->w_elems, al));
    p->xv_elems = int(round_up(p->xv_elems, al));
    std::vector<int64_t> order(static_cast<size_t>(count));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return work[size_t(x)] > work[size_t(y)]; });
    std::vector<CuboidDesc> sorted(static_cast<size_t>(count));
    for (int64_t k = 0; k < count; ++k) sorted[size_t(k)] = desc[size_t(order[size_t(k)])];

    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return TTM_ERR_HIP; }
    p->cu_count = device_cu_count();
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMalloc(reinterpret_cast<void **>(&p->d_desc), sizeof(CuboidDesc) * size_t(count)) != hipSuccess) {
        delete p;
        return TTM_ERR_HIP;
    }
    if (hipMemcpyAsync(p->d_desc, sorted.data(), sizeof(CuboidDesc) * size_t(count), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(p->d_desc);
        delete p;
        return TTM_ERR_HIP;
    }
    const size_t lds_wave = lds_per_wave(p);
    const size_t lds_need = lds_wave * 4;
    if (hipFuncSetAttribute(kernel_ptr(dtype), hipFuncAttributeMaxDynamicSharedMemorySize, int(std::min<size_t>(lds_need, 160 * 1024))) != hipSuccess) {
        (void)hipFree(p->d_desc);
        delete p;
        return TTM_ERR_HIP;
    }
    // default launch shape: 4 waves per block, as many resident blocks as LDS allows (at most 4)
    p->threads = 256;
    while (p->threads > 64 && max_blocks_per_cu(p, p->threads) < 1) p->threads /= 2;
    if (max_blocks_per_cu(p, p->threads) < 1) {
        (void)hipFree(p->d_desc);
        delete p;
        return TTM_ERR_UNSUPPORTED;
    }
    p->blocks_per_cu = std::min(4, max_blocks_per_cu(p, p->threads));

    // workload class for the tuning cache: device, dtype, max sizes, count bucket
    int64_t maxd = 0, sumw = 0;
    for (int64_t k = 0; k < count * 6; ++k) maxd = std::max(maxd, dims_host[k]);
    for (int64_t k = 0; k < count; ++k) sumw += work[size_t(k)];
    char key[256];
    snprintf(key, sizeof key, "%s|%s|maxn%lld|count%lld|work%lld", arch_name().c_str(), dtype == TTM_F64 ? "f64" : "f32",
             (long long)maxd, (long long)count, (long long)(sumw / count));
    p->tune_key = key;
    if (tune_cache) {
        p->tune_cache = tune_cache;
        int t = 0, b = 0;
        if (cache_lookup(p->tune_cache, p->tune_key, t, b) && b <= max_blocks_per_cu(p, t)) {
            p->threads = t;
            p->blocks_per_cu = b;
        }
    }
    *out = p;
    return TTM_OK;
}

int ttm_batched_plan_destroy(ttm_batched_plan *p) {
    if (!p) return TTM_ERR_INVALID_ARG;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_desc) (void)hipFree(p->d_desc);
    delete p;
    return TTM_OK;
}

int ttm_batched_plan_totals(const ttm_batched_plan *p, int64_t *totals) {
    if (!p || !totals) return TTM_ERR_INVALID_ARG;
    for (int n = 0; n < 5; ++n) totals[n] = p->totals[n];
    return TTM_OK;
}

int ttm_batched_plan_config(const ttm_batched_plan *p, int *out) {
    if (!p || !out) return TTM_ERR_INVALID_ARG;
    out[0] = p->threads;
    out[1] = p->blocks_per_cu;
    out[2] = int(std::min<int64_t>(int64_t(p->cu_count) * p->blocks_per_cu, ceil_div(p->count, p->threads / 64)));
    return TTM_OK;
}

int ttm_chain_batched(const ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y,
                      void *stream) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    return launch_batched(p, make_args(p, X, A, B, C, Y), p->threads, p->blocks_per_cu, static_cast<hipStream_t>(stream));
}

int ttm_chain_batched_graph(ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y,
                            void *stream) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    p->graph_args = make_args(p, X, A, B, C, Y);
    p->graph_ptrs[0] = X; p->graph_ptrs[1] = A; p->graph_ptrs[2] = B; p->graph_ptrs[3] = C; p->graph_ptrs[4] = Y;
    p->graph_params[0] = &p->graph_args;
    for (int i = 0; i < 5; ++i) p->graph_params[1 + i] = &p->graph_ptrs[i];
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    int64_t nblocks = int64_t(p->cu_count) * p->blocks_per_cu;
    const int64_t useful = ceil_div(p->count, p->threads / 64);
    if (nblocks > useful) nblocks = useful;
    kp.func = const_cast<void *>(kernel_ptr(p->dtype));
    kp.gridDim = dim3(unsigned(nblocks));
    kp.blockDim = dim3(unsigned(p->threads));
    kp.sharedMemBytes = unsigned(lds_per_wave(p) * size_t(p->threads / 64));
    kp.kernelParams = p->graph_params;
    kp.extra = nullptr;
    if (!p->exec) {
        if (hipGraphCreate(&p->graph, 0) != hipSuccess) return TTM_ERR_HIP;
        if (hipGraphAddKernelNode(&p->node, p->graph, nullptr, 0, &kp) != hipSuccess) return TTM_ERR_HIP;
        if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) return TTM_ERR_HIP;
    } else {
        if (hipGraphExecKernelNodeSetParams(p->exec, p->node, &kp) != hipSuccess) return TTM_ERR_HIP;
    }
    launch_begin("ttm_batched_graph", st);
    hipError_t e = hipGraphLaunch(p->exec, st);
    launch_end(st);
    return e == hipSuccess ? TTM_OK : TTM_ERR_HIP;
}

int ttm_chain_batched_loop(const ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C,
                           void *Y, void *stream) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchArgs a = make_args(p, X, A, B, C, Y);
    a.count = 1;
    const size_t lds = lds_per_wave(p);
    for (int64_t k = 0; k < p->count; ++k) {
        a.desc = p->d_desc + k;
        const bool f64 = p->dtype == TTM_F64;
        if (f64)
            hipLaunchKernelGGL(k_batched<double>, dim3(1), dim3(64), lds, st, a, static_cast<const double *>(X),
                               static_cast<const double *>(A), static_cast<const double *>(B),
                               static_cast<const double *>(C), static_cast<double *>(Y));
        else
            hipLaunchKernelGGL(k_batched<float>, dim3(1), dim3(64), lds, st, a, static_cast<const float *>(X),
                               static_cast<const float *>(A), static_cast<const float *>(B),
                               static_cast<const float *>(C), static_cast<float *>(Y));
        if (hipGetLastError() != hipSuccess) return TTM_ERR_HIP;
    }
    return TTM_OK;
}

int ttm_batched_autotune(ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y,
                         void *stream, int reps, double *best_ms_out) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    if (reps < 1) reps = 1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BatchArgs a = make_args(p, X, A, B, C, Y);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TTM_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return TTM_ERR_HIP; }
    double best = 1e30;
    int bt = p->threads, bb = p->blocks_per_cu;
    const int threads_c[3] = {64, 128, 256};
    const int bpc_c[8] = {1, 2, 3, 4, 6, 8, 12, 16};
    const bool was_timing = timing_on();
    if (was_timing) ttm_timing_enable(0);
    for (int ti = 0; ti < 3 && rc == TTM_OK; ++ti) {
        const int t = threads_c[ti];
        const int maxb = max_blocks_per_cu(p, t);
        for (int bi = 0; bi < 8 && rc == TTM_OK; ++bi) {
            const int b = bpc_c[bi];
            if (b > maxb) continue;
            if ((rc = launch_batched(p, a, t, b, st)) != TTM_OK) break;   // warm-up
            if (hipEventRecord(e0, st) != hipSuccess) { rc = TTM_ERR_HIP; break; }
            for (int r = 0; r < reps && rc == TTM_OK; ++r) rc = launch_batched(p, a, t, b, st);
            if (rc) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = TTM_ERR_HIP; break; }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = TTM_ERR_HIP; break; }
            const double per = double(ms) / reps;
            if (per < best) { best = per; bt = t; bb = b; }
        }
    }
    if (was_timing) ttm_timing_enable(1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    p->threads = bt;
    p->blocks_per_cu = bb;
    if (p->exec) {   // the graph node keeps the old shape: rebuild on next use
        (void)hipGraphExecDestroy(p->exec);
        (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
    if (best_ms_out) *best_ms_out = best;
    if (!p->tune_cache.empty()) cache_store(p->tune_cache, p->tune_key, bt, bb, best);
    return TTM_OK;
}

}  // extern "C"
