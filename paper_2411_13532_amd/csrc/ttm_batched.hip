// ttm_batched.hip -- many small independent chains Y_k = X_k x1 A_k x2 B_k x3 C_k
// (ragged sizes, every mode at most 16) in one persistent launch.
//
// One wavefront owns one cuboid at a time and its lanes own fibers, as the
// paper maps independent lines onto the lanes of one execution unit (Sec.
// 4.1, the SZ-grouped layout).  Each mode product is a loop over fibers of
// the current intermediate, one fiber per lane (64 per pass, at most four
// passes): the lane holds the fiber's values in registers and forms every
// output of that fiber as a dot product with a factor row, which all lanes
// read from LDS at the same address (a broadcast, 16 bytes at a time).
//   mode 3: fibers (i1, i2) of X along i3     -> W[i1][i2][j3]
//   mode 2: fibers (i1, j3) of W along i2     -> V[i1][j2][j3]
//   mode 1: fibers (j2, j3) of V along i1     -> Y[j1][j2][j3]
// One LDS region per wave holds X, then W, then V (each pass reads all its
// fibers into registers before the region is overwritten), and one factor
// region holds the factor of the current mode (the cuboid's three factors
// wait in registers, at most four elements per lane each): at n <= 13 about
// 9.6 KiB per wave, so that four waves per SIMD fit in LDS.  X is read
// from HBM with coalesced loads of the whole cuboid and scattered to fibers
// at odd strides (no bank conflicts); Y is written with coalesced stores.
// The next cuboid's X and factors are loaded into registers while the wave
// works on the current one.
//
// The matrix-core variants (MX) form each mode product as 16 x 16 x 4 float
// products instead (mode_mfma): the factor is the A operand, held in
// registers, and 16 fibers form the B operand of each tile, read from the
// same LDS region.  Lanes whose output falls outside the result store it to
// a dump slot in the (unused) factor region instead of being masked off, and
// Y is assembled in the region in its own layout and then stored in whole
// 256-byte rows (the region holds J1 J2 J3 values too).  The wave's time per
// cuboid is mostly the latency and issue of its dependent steps (load X,
// three products, store Y); the kernel runs as fast as resident waves allow.
//
// Work assignment: the plan sorts the cuboids longest first and deals them
// to the waves of the launch by LPT (each to the wave with the least work so
// far, by a cost model of the passes and dot products above plus a fixed
// term per cuboid for its chain of dependent steps); wave w runs
// its list desc[start[w] .. start[w + 1]).  The launch shape (threads per
// block, resident blocks per compute unit) is autotuned per workload on a
// cold last-level cache and cached; the assignment follows the shape.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <utility>
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
    const CuboidDesc *desc;       // in processing order
    const int32_t *wave_start;    // per wave: first entry of its list (total waves + 1), or null
    int64_t count;
    int fac_elems, buf_elems;     // per-wave LDS regions (elements)
};

// X of the next cuboid is loaded into registers (BATCH_PF elements per lane,
// every load issued before any is used) while the wave works on the current
// one; a larger X loads its rest at stage 0.
constexpr int BATCH_PF = 16;

// fixed part of a cuboid's cost in the work assignment (units of the
// per-mode pass x group x group terms)
constexpr double BATCH_CUBOID_COST = 100.0;

// Row r = e / len for e < 4096, len <= 16: the float quotient is at least
// 1/32 away from the next integer, far more than its rounding error (also
// with the hardware reciprocal, 1 ulp).
__device__ __forceinline__ int row_of(int e, float inv_len) { return int((float(e) + 0.5f) * inv_len); }

// n (<= 256) elements of a factor (rows of len), already loaded as
// r[u] = element u * 64 + lane, into LDS rows of stride P, and zeros into the
// P - len (< 4) padding columns of its n / len rows (the dot products read
// them against zero fiber values: they must be finite).
template <typename T>
__device__ __forceinline__ void factor_regs_to_lds(const T (&r)[4], int n, int len, int P, T *dst, int lane) {
    const float inv = __builtin_amdgcn_rcpf(float(len));
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = u * 64 + lane;
        const int row = row_of(e, inv);
        if (e < n) dst[row * P + (e - row * len)] = r[u];
    }
    const int pad = P - len, rows = n / len;
    if (pad > 0 && lane < rows * pad) {
        const int row = lane / pad;
        dst[row * P + len + (lane - row * pad)] = T(0);
    }
}

// One mode product of a cuboid, a lane per fiber: NF fibers (NP passes of
// 64 lanes; fiber p * 64 + lane in pass p) of length L (L4 groups of 4), M
// outputs per fiber: out[obase(f) + j * ostride] = sum_{e < L} U[j][e] x_f[e]
// with x_f[e] = buf[rbase(f) + e * rstride].  Every pass's fibers are read
// into registers before any output is written, so the outputs may overwrite
// the fibers (the caller syncs the wave before and after).  The factor U is
// in LDS rows of stride P (a multiple of 4, zero-padded past L, plus three
// spare rows past M); four rows of four values are read at a time, at the
// same address on every lane (a broadcast), and shared by all passes.  Fixed
// order of the terms.  (Specialising on L itself instead of L4 removes the
// padded terms but multiplies the code: measured slower, the hot code no
// longer fits the instruction cache.)
template <int L4, int NP, typename T, typename RB, typename OB>
__device__ __forceinline__ void mode_body(const T *buf, int NF, int L, const T *U, int P, int M, RB rbase,
                                          int rstride, T *lout, T *gout, OB obase, int ostride, int lane) {
    typedef T T4 __attribute__((ext_vector_type(4)));
    T fv[NP][4 * L4];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int f = p * 64 + lane < NF ? p * 64 + lane : NF - 1;   // spare lanes read a valid fiber
        const int b = rbase(f);
#pragma unroll
        for (int e = 0; e < 4 * L4; ++e) {
            const int ec = e < L ? e : L - 1;                            // uniform
            const T v = buf[b + ec * rstride];
            fv[p][e] = e < L ? v : T(0);
        }
    }
    wave_sync();   // every fiber is in registers: the outputs may overwrite them
    for (int j = 0; j < M; j += 4) {
        T acc[NP][4];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[p][r] = T(0);
#pragma unroll
        for (int e4 = 0; e4 < L4; ++e4) {
            T4 u[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = *reinterpret_cast<const T4 *>(U + (j + r) * P + 4 * e4);
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[p][r] += u[r][i] * fv[p][4 * e4 + i];
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int f = p * 64 + lane;
            if (f < NF) {
                const int64_t o = obase(f) + int64_t(j) * ostride;
                if (gout) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j + r < M) gout[o + int64_t(r) * ostride] = acc[p][r];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (j + r < M) lout[o + r * ostride] = acc[p][r];
                }
            }
        }
    }
}

// mode_body for runtime L (1..16) and NF (1..256); outputs go to global
// memory gout when it is not null, else to LDS lout
template <typename T, typename RB, typename OB>
__device__ __forceinline__ void mode_any(const T *buf, int NF, int L, const T *U, int P, int M, RB rbase, int rstride,
                                         T *lout, T *gout, OB obase, int ostride, int lane) {
    const int L4 = (L + 3) >> 2, NP = (NF + 63) >> 6;
#define TTM_MODE_CASE(l4, np)                                                                             \
    case (l4 - 1) * 4 + (np - 1):                                                                         \
        mode_body<l4, np>(buf, NF, L, U, P, M, rbase, rstride, lout, gout, obase, ostride, lane);         \
        break;
    switch ((L4 - 1) * 4 + (NP - 1)) {
        TTM_MODE_CASE(1, 1) TTM_MODE_CASE(1, 2) TTM_MODE_CASE(1, 3) TTM_MODE_CASE(1, 4)
        TTM_MODE_CASE(2, 1) TTM_MODE_CASE(2, 2) TTM_MODE_CASE(2, 3) TTM_MODE_CASE(2, 4)
        TTM_MODE_CASE(3, 1) TTM_MODE_CASE(3, 2) TTM_MODE_CASE(3, 3) TTM_MODE_CASE(3, 4)
        TTM_MODE_CASE(4, 1) TTM_MODE_CASE(4, 2) TTM_MODE_CASE(4, 3) TTM_MODE_CASE(4, 4)
        default: break;
    }
#undef TTM_MODE_CASE
}

// One mode product on the matrix cores (float): D[j][f] = sum_{k < L}
// U[j][k] x_f[k] for j < M (<= 16) and fibers f < NF (<= 16 * NTM) of length
// L (<= 4 * KS), as 16 x 16 x 4 products, one 16-fiber tile per accumulator.
// The factor is the A operand: lane l holds row l % 16 and the k slots
// (l / 16) * KS + s in ua[s] (zero past M and L).  The fibers are the B
// operand: column l % 16 of tile t is fiber 16 t + l % 16, its k slots read
// from buf[rbase(f) + k * rstride], the fiber and k clamped to valid elements
// where the factor slot is zero (the value only has to be finite).  Lane l's
// accumulator element r is D[4 (l / 16) + r][16 t + l % 16], written to
// out[obase(f) + j * ostride] in LDS; lanes past NF or M write out[dump]
// instead (a slot nothing reads), so no store is masked.  Every tile is
// formed before any output is written, so the outputs may overwrite the
// fibers (the caller syncs the wave before and after).  Fixed order of the
// terms.
template <int KS, int NTM, typename RB, typename OB>
__device__ __forceinline__ void mode_mfma_body(const float *buf, int NF, int L, const float (&ua)[4], int M, RB rbase,
                                               int rstride, float *out, OB obase, int ostride, int dump, int lane) {
    const int c = lane & 15, g = lane >> 4;
    const int NT = (NF + 15) >> 4;
    int kofs[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int k = g * KS + s;
        kofs[s] = (k < L ? k : L - 1) * rstride;
    }
    f32x4 acc[NTM];
#pragma unroll
    for (int t = 0; t < NTM; ++t) {
        if (t < NT) {   // uniform
            const int f = t * 16 + c;
            const int b = rbase(f < NF ? f : NF - 1);
            float x[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) x[s] = buf[b + kofs[s]];
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc[t] = mfma_f32(ua[s], x[s], acc[t]);
        }
    }
    wave_sync();   // every tile is formed: the outputs may overwrite the fibers
#pragma unroll
    for (int t = 0; t < NTM; ++t) {
        if (t < NT) {   // uniform
            const int f = t * 16 + c;
            const int o = obase(f < NF ? f : NF - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 4 * g + r;
                out[f < NF && j < M ? o + j * ostride : dump] = acc[t][r];
            }
        }
    }
}

// mode_mfma_body for runtime L (1..16) and NF (1..256)
template <typename RB, typename OB>
__device__ __forceinline__ void mode_mfma(const float *buf, int NF, int L, const float (&ua)[4], int M, RB rbase,
                                          int rstride, float *out, OB obase, int ostride, int dump, int lane) {
    const int KS = (L + 3) >> 2, NTQ = (NF + 63) >> 6;
#define TTM_MX_CASE(ks, ntq)                                                                              \
    case (ks - 1) * 4 + (ntq - 1):                                                                        \
        mode_mfma_body<ks, 4 * ntq>(buf, NF, L, ua, M, rbase, rstride, out, obase, ostride, dump, lane);  \
        break;
    switch ((KS - 1) * 4 + (NTQ - 1)) {
        TTM_MX_CASE(1, 1) TTM_MX_CASE(1, 2) TTM_MX_CASE(1, 3) TTM_MX_CASE(1, 4)
        TTM_MX_CASE(2, 1) TTM_MX_CASE(2, 2) TTM_MX_CASE(2, 3) TTM_MX_CASE(2, 4)
        TTM_MX_CASE(3, 1) TTM_MX_CASE(3, 2) TTM_MX_CASE(3, 3) TTM_MX_CASE(3, 4)
        TTM_MX_CASE(4, 1) TTM_MX_CASE(4, 2) TTM_MX_CASE(4, 3) TTM_MX_CASE(4, 4)
        default: break;
    }
#undef TTM_MX_CASE
}

// OCC: resident waves per SIMD the register budget is cut for (a launch
// variant the autotuner chooses).  At two, the next cuboid's first
// BATCH_PF * 64 elements of X and its factors are loaded into registers while
// the wave works on the current one (with MX at three, half as many rows of
// X); otherwise there is no room for that, and the other resident waves
// cover the load latency instead.
// MX: the mode products on the matrix cores (mode_mfma, float only); the
// factors then stay in registers in the A-operand layout and the LDS factor
// region is unused.
template <typename T, int OCC, bool MX = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC)))
k_batched(const BatchArgs a, const T *__restrict__ X, const T *__restrict__ Ag, const T *__restrict__ Bg,
          const T *__restrict__ Cg, T *__restrict__ Y) {
    constexpr int PF = OCC <= 2 ? BATCH_PF : MX && OCC == 3 ? BATCH_PF / 2 : 0;
    constexpr int PFF = PF > 0 ? 4 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int wpb = blockDim.x >> 6;
    T *fac = reinterpret_cast<T *>(smem_raw) + int64_t(wave) * (a.fac_elems + a.buf_elems);
    T *buf = fac + a.fac_elems;
    const int64_t gw = int64_t(blockIdx.x) * wpb + wave;
    int64_t k0, k1, kstep;
    if (a.wave_start) {
        k0 = a.wave_start[gw];
        k1 = a.wave_start[gw + 1];
        kstep = 1;
    } else {
        k0 = gw;
        k1 = a.count;
        kstep = int64_t(gridDim.x) * wpb;
    }

    // the first PF rows of 64 elements of a cuboid's X and its three factors
    // (at most 256 elements each, 4 per lane); fr: the current cuboid's
    // factors until their modes
    static_assert(!MX || std::is_same<T, float>::value, "matrix-core variant is float only");
    T pre[PF > 0 ? PF : 1], pf[3][4], fr[3][4];
    // a factor U (J x I) into four registers per lane: elements u * 64 + lane
    // (rows of 64 the factor fills), or with MX the A-operand slots of
    // mode_mfma (row lane % 16, k = (lane / 16) * KS + s, zero elsewhere)
    auto load_factor = [&](const T *U, int J, int I, T (&dst)[4]) __attribute__((always_inline)) {
        if constexpr (MX) {
            const int c = lane & 15, g = lane >> 4, KS = (I + 3) >> 2;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = g * KS + s;
                dst[s] = (c < J && s < KS && k < I) ? U[c * I + k] : T(0);
            }
        } else {
            const int n = J * I;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = u * 64 + lane;
                if (u * 64 < n) dst[u] = U[e < n ? e : n - 1];   // uniform: rows of 64 the factor fills
            }
        }
    };
    auto load_inputs = [&](const CuboidDesc &d) __attribute__((always_inline)) {
        const int nx = d.d[0] * d.d[1] * d.d[2];
        const T *xs = X + d.ox;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            if (u * 64 < nx) {   // uniform: only the rows of 64 that X fills
                const int e = u * 64 + lane;
                pre[u] = xs[e < nx ? e : nx - 1];
            }
        }
        if constexpr (PF > 0) {
            const T *fs[3] = {Ag + d.oa, Bg + d.ob, Cg + d.oc};
#pragma unroll
            for (int f = 0; f < 3; ++f) load_factor(fs[f], d.d[3 + f], d.d[f], pf[f]);
        }
    };
    auto prefetch = [&](const CuboidDesc &d) __attribute__((always_inline)) {
        if constexpr (PF > 0) load_inputs(d);
    };

    if (k0 < k1) prefetch(a.desc[k0]);
    for (int64_t k = k0; k < k1; k += kstep) {
        const CuboidDesc d = a.desc[k];
        const int I1 = d.d[0], I2 = d.d[1], I3 = d.d[2], J1 = d.d[3], J2 = d.d[4], J3 = d.d[5];
        // factor rows padded to multiples of 4 (zeros); odd strides for fibers
        const int P1 = (I1 + 3) & ~3, P2 = (I2 + 3) & ~3, P3 = (I3 + 3) & ~3;
        const int nx = I1 * I2 * I3;

        // stage 0: the factors into registers (prefetched, or loaded now),
        // C into the zero-padded LDS factor rows, X (prefetched, plus any
        // rest) into fibers of odd stride SX
        if constexpr (PF > 0) {
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int u = 0; u < 4; ++u) fr[f][u] = pf[f][u];
        } else {
            const T *fs[3] = {Ag + d.oa, Bg + d.ob, Cg + d.oc};
            if constexpr (MX) {
#pragma unroll
                for (int f = 0; f < 3; ++f) load_factor(fs[f], d.d[3 + f], d.d[f], fr[f]);
            } else {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int n = d.d[3 + f] * d.d[f];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = u * 64 + lane;
                        if (u * 64 < n) fr[f][u] = fs[f][e < n ? e : n - 1];   // uniform: rows of 64 the factor fills
                    }
                }
            }
        }
        if constexpr (!MX) factor_regs_to_lds(fr[2], J3 * I3, I3, P3, fac, lane);
        const int SX = I3 | 1;
        const float inv3 = __builtin_amdgcn_rcpf(float(I3));
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            if (u * 64 < nx) {
                const int e = u * 64 + lane;
                const int f = row_of(e, inv3);
                if (e < nx) buf[f * SX + (e - f * I3)] = pre[u];
            }
        }
        for (int base = PF * 64; base < nx; base += 16 * 64) {
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
                if constexpr (MX) buf[e < nx ? f * SX + (e - f * I3) : -a.fac_elems] = r[u];   // past X: dump slot
                else if (e < nx) buf[f * SX + (e - f * I3)] = r[u];
            }
        }
        wave_sync();
        if (k + kstep < k1) prefetch(a.desc[k + kstep]);

        // mode 3: fiber f = (i1, i2) along i3 -> W[f][j3] at row stride SW
        const int SW = J3 | 1;
        auto rb3 = [&](int f) { return f * SX; };
        auto ob3 = [&](int f) { return f * SW; };
        if constexpr (MX) mode_mfma(buf, I1 * I2, I3, fr[2], J3, rb3, 1, buf, ob3, 1, -a.fac_elems, lane);
        else mode_any(buf, I1 * I2, I3, fac, P3, J3, rb3, 1, buf, static_cast<T *>(nullptr), ob3, 1, lane);
        wave_sync();
        if constexpr (!MX) {
            factor_regs_to_lds(fr[1], J2 * I2, I2, P2, fac, lane);
            wave_sync();
        }
        // mode 2: fiber g = (i1, j3) along i2 -> V[i1][j2][j3] at i1 stride SV
        const int SV = (J2 * J3) | 1;
        const float invJ3 = __builtin_amdgcn_rcpf(float(J3));
        auto rb2 = [&](int g) { const int i1 = row_of(g, invJ3); return i1 * I2 * SW + (g - i1 * J3); };
        auto ob2 = [&](int g) { const int i1 = row_of(g, invJ3); return i1 * SV + (g - i1 * J3); };
        if constexpr (MX) mode_mfma(buf, I1 * J3, I2, fr[1], J2, rb2, SW, buf, ob2, J3, -a.fac_elems, lane);
        else mode_any(buf, I1 * J3, I2, fac, P2, J2, rb2, SW, buf, static_cast<T *>(nullptr), ob2, J3, lane);
        wave_sync();
        if constexpr (!MX) {
            factor_regs_to_lds(fr[0], J1 * I1, I1, P1, fac, lane);
            wave_sync();
        }
        // mode 1: fiber h = (j2, j3) along i1 -> Y[j1][h]
        const int H = J2 * J3;
        auto rb1 = [&](int h) { return h; };
        if constexpr (MX) {
            // Y in its own layout [j1][h] into the region (every tile is
            // formed before the region is written), then out with whole
            // 256-byte rows of stores
            mode_mfma(buf, H, I1, fr[0], J1, rb1, SV, buf, rb1, H, -a.fac_elems, lane);
            wave_sync();
            const int ny = J1 * H;
            T *ys = Y + d.oy;
#pragma unroll 4
            for (int e = lane; e < ny; e += 64) ys[e] = buf[e];
        } else {
            mode_any(buf, H, I1, fac, P1, J1, rb1, SV, buf, Y + d.oy, rb1, H, lane);
        }
        wave_sync();
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
    std::vector<CuboidDesc> desc;      // input order
    std::vector<double> cost;          // cost model per cuboid (input order)
    std::vector<int64_t> by_cost;      // cuboid indices, longest first
    CuboidDesc *d_desc = nullptr;      // processing order of the current assignment
    int32_t *d_start = nullptr;        // per wave: first entry of its list (+ end)
    int64_t assigned_waves = 0;        // waves the device lists were built for
    int fac_elems = 0, buf_elems = 0;
    int threads = 256, blocks_per_cu = 2, variant = 1;
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

size_t lds_per_wave(const ttm_batched_plan *p) { return size_t(p->fac_elems + p->buf_elems) * p->esz; }

// resident waves per SIMD the register budget of a launch variant allows
int variant_occupancy(int dtype, int variant) {
    if (dtype == TTM_F64) return 1;
    return variant < 3 ? variant + 2 : variant == 3 ? 3 : 4;
}

int max_blocks_per_cu(const ttm_batched_plan *p, int threads, int variant) {
    const size_t per_block = lds_per_wave(p) * size_t(threads / 64);
    const size_t lds_cu = 160 * 1024;
    int b = int(lds_cu / std::max<size_t>(per_block, 1));
    const int waves_cap = 4 * variant_occupancy(p->dtype, variant) / (threads / 64);   // resident per CU
    return std::max(0, std::min(b, waves_cap));
}

int64_t launch_waves(const ttm_batched_plan *p, int threads, int bpc) {
    int64_t nblocks = int64_t(p->cu_count) * bpc;
    const int64_t useful = ceil_div(p->count, threads / 64);
    if (nblocks > useful) nblocks = useful;
    if (nblocks < 1) nblocks = 1;
    return nblocks * (threads / 64);
}

// LPT over `waves` workers: cuboids longest first, each to the wave with the
// least work so far (ties to the lowest wave index); the device gets the
// cuboids grouped by wave, in the order each wave takes them, and the start
// of every wave's run.  Synchronous (plan creation and autotuning only).
int assign_waves(ttm_batched_plan *p, int64_t waves, hipStream_t st) {
    if (p->assigned_waves == waves) return TTM_OK;
    typedef std::pair<double, int64_t> Load;   // (work, wave)
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int64_t w = 0; w < waves; ++w) heap.push(Load(0.0, w));
    std::vector<int64_t> owner(size_t(p->count));
    std::vector<int32_t> start(size_t(waves) + 1, 0);
    for (int64_t k : p->by_cost) {
        Load l = heap.top();
        heap.pop();
        owner[size_t(k)] = l.second;
        start[size_t(l.second) + 1] += 1;
        l.first += p->cost[size_t(k)];
        heap.push(l);
    }
    for (int64_t w = 0; w < waves; ++w) start[size_t(w) + 1] += start[size_t(w)];
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    std::vector<CuboidDesc> ordered(size_t(p->count));
    for (int64_t k : p->by_cost) ordered[size_t(fill[size_t(owner[size_t(k)])]++)] = p->desc[size_t(k)];
    if (p->d_start) { (void)hipFree(p->d_start); p->d_start = nullptr; }
    if (hipMalloc(reinterpret_cast<void **>(&p->d_start), sizeof(int32_t) * size_t(waves + 1)) != hipSuccess)
        return TTM_ERR_HIP;
    if (hipMemcpyAsync(p->d_desc, ordered.data(), sizeof(CuboidDesc) * size_t(p->count), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(p->d_start, start.data(), sizeof(int32_t) * size_t(waves + 1), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return TTM_ERR_HIP;
    p->assigned_waves = waves;
    return TTM_OK;
}

BatchArgs make_args(const ttm_batched_plan *p) {
    BatchArgs a;
    a.desc = p->d_desc;
    a.wave_start = p->d_start;
    a.count = p->count;
    a.fac_elems = p->fac_elems;
    a.buf_elems = p->buf_elems;
    return a;
}

// Launch variants: the register budget of k_batched (resident waves per
// SIMD) and where the mode products run.  float: 0, 1, 2 on the vector units
// at 2 (with register prefetch of the next cuboid), 3 or 4 waves per SIMD;
// 3 and 4 on the matrix cores at 3 (prefetching the next cuboid's factors and
// first 512 elements of X) or 4.  double: one kernel (1 wave per SIMD, vector
// units) for every variant.
constexpr int BATCH_VARIANTS = 5;
const void *kernel_ptr(int dtype, int variant) {
    if (dtype == TTM_F64)
        return reinterpret_cast<const void *>(&k_batched<double, 1>);
    switch (variant) {
        case 0: return reinterpret_cast<const void *>(&k_batched<float, 2>);
        case 1: return reinterpret_cast<const void *>(&k_batched<float, 3>);
        case 2: return reinterpret_cast<const void *>(&k_batched<float, 4>);
        case 3: return reinterpret_cast<const void *>(&k_batched<float, 3, true>);
        default: return reinterpret_cast<const void *>(&k_batched<float, 4, true>);
    }
}
template <typename T>
void launch_variant(int variant, dim3 grid, dim3 block, size_t lds, hipStream_t st, const BatchArgs &a, const void *X,
                    const void *A, const void *B, const void *C, void *Y) {
    const T *x = static_cast<const T *>(X), *pa = static_cast<const T *>(A), *pb = static_cast<const T *>(B),
            *pc = static_cast<const T *>(C);
    T *y = static_cast<T *>(Y);
    constexpr bool F = std::is_same<T, float>::value;
    if (variant == 0 || !F) hipLaunchKernelGGL((k_batched<T, F ? 2 : 1>), grid, block, lds, st, a, x, pa, pb, pc, y);
    else if (variant == 1) hipLaunchKernelGGL((k_batched<T, F ? 3 : 1>), grid, block, lds, st, a, x, pa, pb, pc, y);
    else if (variant == 2) hipLaunchKernelGGL((k_batched<T, F ? 4 : 1>), grid, block, lds, st, a, x, pa, pb, pc, y);
    else if (variant == 3) hipLaunchKernelGGL((k_batched<T, F ? 3 : 1, F>), grid, block, lds, st, a, x, pa, pb, pc, y);
    else hipLaunchKernelGGL((k_batched<T, F ? 4 : 1, F>), grid, block, lds, st, a, x, pa, pb, pc, y);
}

// One launch of the persistent kernel with the plan's current assignment
// (threads per block must be the one it was built for).
int launch_batched(const ttm_batched_plan *p, const BatchArgs &a, const void *X, const void *A, const void *B,
                   const void *C, void *Y, int threads, int variant, hipStream_t st) {
    const size_t lds = lds_per_wave(p) * size_t(threads / 64);
    const int64_t nblocks = p->assigned_waves / (threads / 64);
    return launch("ttm_batched", st, [&] {
        if (p->dtype == TTM_F64)
            launch_variant<double>(variant, dim3(unsigned(nblocks)), dim3(threads), lds, st, a, X, A, B, C, Y);
        else
            launch_variant<float>(variant, dim3(unsigned(nblocks)), dim3(threads), lds, st, a, X, A, B, C, Y);
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
//   "<key>": {"threads": T, "blocks_per_cu": B, "variant": V, "ms": M},
//   ...
//   }
bool cache_lookup(const std::string &path, const std::string &key, int &threads, int &bpc, int &variant) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string needle = "\"" + key + "\":";
    while (fgets(line, sizeof line, f)) {
        if (strstr(line, needle.c_str()) != line) continue;
        const char *t = strstr(line, "\"threads\":");
        const char *b = strstr(line, "\"blocks_per_cu\":");
        const char *v = strstr(line, "\"variant\":");
        if (t && b && v) {
            threads = atoi(t + 10);
            bpc = atoi(b + 16);
            variant = atoi(v + 10);
            found = (threads == 64 || threads == 128 || threads == 256) && variant >= 0 && variant < BATCH_VARIANTS;
        }
        break;
    }
    fclose(f);
    return found && bpc >= 1;
}

bool cache_store(const std::string &path, const std::string &key, int threads, int bpc, int variant, double ms) {
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
    snprintf(buf, sizeof buf, "\"%s\": {\"threads\": %d, \"blocks_per_cu\": %d, \"variant\": %d, \"ms\": %.6f}",
             key.c_str(), threads, bpc, variant, ms);
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
    if (count > (int64_t(1) << 31) - 1) return TTM_ERR_UNSUPPORTED;
    for (int64_t k = 0; k < count * 6; ++k)
        if (dims_host[k] < 1 || dims_host[k] > BATCH_MAXN) return TTM_ERR_INVALID_ARG;

    ttm_batched_plan *p = new ttm_batched_plan();
    p->count = count;
    p->dtype = dtype;
    p->esz = dtype == TTM_F64 ? 8 : 4;
    p->dims.assign(dims_host, dims_host + count * 6);

    // offsets in input order; per-wave LDS for the largest cuboid; the cost
    // model: per mode, passes of 64 fibers x groups of 4 along the fiber x
    // groups of 4 outputs, plus the load of X, plus a fixed term for the
    // cuboid's chain of dependent steps (load, three products, store), whose
    // latency a wave pays per cuboid whatever its size: without it, waves
    // dealt many small cuboids finish last (measured: any fixed term from 80
    // up balances the same, 4 % faster than none)
    p->desc.resize(size_t(count));
    p->cost.resize(size_t(count));
    int64_t o[5] = {0, 0, 0, 0, 0};
    for (int64_t k = 0; k < count; ++k) {
        const int64_t *d = dims_host + 6 * k;
        CuboidDesc &c = p->desc[size_t(k)];
        c.ox = o[0]; c.oa = o[1]; c.ob = o[2]; c.oc = o[3]; c.oy = o[4];
        for (int n = 0; n < 6; ++n) c.d[n] = int32_t(d[n]);
        o[0] += d[0] * d[1] * d[2];
        o[1] += d[3] * d[0];
        o[2] += d[4] * d[1];
        o[3] += d[5] * d[2];
        o[4] += d[3] * d[4] * d[5];
        auto g4 = [](int64_t v) { return double(ceil_div(v, 4)); };
        auto ps = [](int64_t v) { return double(ceil_div(v, 64)); };
        p->cost[size_t(k)] = ps(d[0] * d[1]) * g4(d[2]) * g4(d[5]) + ps(d[0] * d[5]) * g4(d[1]) * g4(d[4]) +
                             ps(d[4] * d[5]) * g4(d[0]) * g4(d[3]) + double(ceil_div(d[0] * d[1] * d[2], 64)) +
                             BATCH_CUBOID_COST;
        p->fac_elems = std::max<int>(p->fac_elems, int(std::max({d[3] * round_up(d[0], 4), d[4] * round_up(d[1], 4),
                                                                  d[5] * round_up(d[2], 4)})));
        p->buf_elems = std::max<int>(p->buf_elems, int(std::max({d[0] * d[1] * (d[2] | 1), d[0] * d[1] * (d[5] | 1),
                                                                  d[0] * ((d[4] * d[5]) | 1), d[3] * d[4] * d[5]})));
    }
    for (int n = 0; n < 5; ++n) p->totals[n] = o[n];
    // the dot products read up to three rows (of at most 16) past a factor's last
    p->fac_elems += 3 * BATCH_MAXN;
    // keep every region 16-byte aligned
    const int al = int(16 / p->esz);
    p->fac_elems = int(round_up(p->fac_elems, al));
    p->buf_elems = int(round_up(p->buf_elems, al));
    p->by_cost.resize(size_t(count));
    std::iota(p->by_cost.begin(), p->by_cost.end(), 0);
    std::stable_sort(p->by_cost.begin(), p->by_cost.end(),
                     [&](int64_t x, int64_t y) { return p->cost[size_t(x)] > p->cost[size_t(y)]; });

    auto fail = [&](int rc) {
        if (p->d_desc) (void)hipFree(p->d_desc);
        if (p->d_start) (void)hipFree(p->d_start);
        delete p;
        return rc;
    };
    if (hipGetDevice(&p->device) != hipSuccess) return fail(TTM_ERR_HIP);
    p->cu_count = device_cu_count();
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMalloc(reinterpret_cast<void **>(&p->d_desc), sizeof(CuboidDesc) * size_t(count)) != hipSuccess)
        return fail(TTM_ERR_HIP);
    const size_t lds_need = lds_per_wave(p) * 4;
    static std::atomic<uint64_t> attr_set[2][BATCH_VARIANTS];
    for (int v = 0; v < BATCH_VARIANTS; ++v)
        if (ensure_lds_limit(kernel_ptr(dtype, v), std::min<size_t>(lds_need, 160 * 1024),
                             attr_set[dtype == TTM_F64][v]))
            return fail(TTM_ERR_HIP);
    // default launch shape: the higher-occupancy variant, 4 waves per block,
    // as many resident blocks as LDS and registers allow
    p->variant = 1;
    p->threads = 256;
    while (p->threads > 64 && max_blocks_per_cu(p, p->threads, p->variant) < 1) p->threads /= 2;
    if (max_blocks_per_cu(p, p->threads, p->variant) < 1) return fail(TTM_ERR_UNSUPPORTED);
    p->blocks_per_cu = max_blocks_per_cu(p, p->threads, p->variant);

    // workload class for the tuning cache: device, dtype, max sizes, count, mean cost
    int64_t maxd = 0;
    double sumc = 0.0;
    for (int64_t k = 0; k < count * 6; ++k) maxd = std::max(maxd, dims_host[k]);
    for (int64_t k = 0; k < count; ++k) sumc += p->cost[size_t(k)];
    char key[256];
    snprintf(key, sizeof key, "%s|%s|v4|maxn%lld|count%lld|cost%lld", arch_name().c_str(),
             dtype == TTM_F64 ? "f64" : "f32", (long long)maxd, (long long)count, (long long)(sumc / count * 100));
    p->tune_key = key;
    if (tune_cache) {
        p->tune_cache = tune_cache;
        int t = 0, b = 0, v = 0;
        if (cache_lookup(p->tune_cache, p->tune_key, t, b, v) && b <= max_blocks_per_cu(p, t, v)) {
            p->threads = t;
            p->blocks_per_cu = b;
            p->variant = v;
        }
    }
    if (int rc = assign_waves(p, launch_waves(p, p->threads, p->blocks_per_cu), st)) return fail(rc);
    *out = p;
    return TTM_OK;
}

int ttm_batched_plan_destroy(ttm_batched_plan *p) {
    if (!p) return TTM_ERR_INVALID_ARG;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_desc) (void)hipFree(p->d_desc);
    if (p->d_start) (void)hipFree(p->d_start);
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
    out[2] = int(p->assigned_waves / (p->threads / 64));
    out[3] = p->variant;
    return TTM_OK;
}

int ttm_batched_plan_set_config(ttm_batched_plan *p, int threads, int blocks_per_cu, int variant, void *stream) {
    if (!p || (threads != 64 && threads != 128 && threads != 256) || variant < 0 || variant >= BATCH_VARIANTS ||
        blocks_per_cu < 1 || blocks_per_cu > max_blocks_per_cu(p, threads, variant))
        return TTM_ERR_INVALID_ARG;
    if (int rc = assign_waves(p, launch_waves(p, threads, blocks_per_cu), static_cast<hipStream_t>(stream))) return rc;
    p->threads = threads;
    p->blocks_per_cu = blocks_per_cu;
    p->variant = variant;
    if (p->exec) {   // the graph node keeps the old shape: rebuild on next use
        (void)hipGraphExecDestroy(p->exec);
        (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
    return TTM_OK;
}

int ttm_chain_batched(const ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y,
                      void *stream) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    return launch_batched(p, make_args(p), X, A, B, C, Y, p->threads, p->variant, static_cast<hipStream_t>(stream));
}

int ttm_chain_batched_graph(ttm_batched_plan *p, const void *X, const void *A, const void *B, const void *C, void *Y,
                            void *stream) {
    int rc = check_buffers(p, X, A, B, C, Y);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    p->graph_args = make_args(p);
    p->graph_ptrs[0] = X; p->graph_ptrs[1] = A; p->graph_ptrs[2] = B; p->graph_ptrs[3] = C; p->graph_ptrs[4] = Y;
    p->graph_params[0] = &p->graph_args;
    for (int i = 0; i < 5; ++i) p->graph_params[1 + i] = &p->graph_ptrs[i];
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    kp.func = const_cast<void *>(kernel_ptr(p->dtype, p->variant));
    kp.gridDim = dim3(unsigned(p->assigned_waves / (p->threads / 64)));
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
    BatchArgs a = make_args(p);
    a.wave_start = nullptr;   // one wave, one cuboid per launch
    a.count = 1;
    const size_t lds = lds_per_wave(p);
    for (int64_t k = 0; k < p->count; ++k) {
        a.desc = p->d_desc + k;
        const bool f64 = p->dtype == TTM_F64;
        if (f64)
            hipLaunchKernelGGL((k_batched<double, 1>), dim3(1), dim3(64), lds, st, a, static_cast<const double *>(X),
                               static_cast<const double *>(A), static_cast<const double *>(B),
                               static_cast<const double *>(C), static_cast<double *>(Y));
        else
            hipLaunchKernelGGL((k_batched<float, 2>), dim3(1), dim3(64), lds, st, a, static_cast<const float *>(X),
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
    // every timed launch starts on a cold last-level cache: a 512 MiB buffer
    // is rewritten before it (the 256 MB cache would otherwise hold a whole
    // batch of this size)
    const size_t flush_bytes = size_t(512) << 20;
    void *flush = nullptr;
    if (hipMalloc(&flush, flush_bytes) != hipSuccess) return TTM_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) { (void)hipFree(flush); return TTM_ERR_HIP; }
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); (void)hipFree(flush); return TTM_ERR_HIP; }
    double best = 1e30;
    int bt = p->threads, bb = p->blocks_per_cu, bv = p->variant;
    const int threads_c[3] = {64, 128, 256};
    const int bpc_c[9] = {1, 2, 3, 4, 6, 8, 12, 16, 24};
    const bool was_timing = timing_on();
    if (was_timing) ttm_timing_enable(0);
    const int nvar = p->dtype == TTM_F64 ? 1 : BATCH_VARIANTS;   // double: one kernel for every variant
    for (int v = 0; v < nvar && rc == TTM_OK; ++v) {
        for (int ti = 0; ti < 3 && rc == TTM_OK; ++ti) {
            const int t = threads_c[ti];
            const int maxb = max_blocks_per_cu(p, t, v);
            for (int bi = 0; bi < 9 && rc == TTM_OK; ++bi) {
                const int b = bpc_c[bi];
                if (b > maxb) continue;
                if ((rc = assign_waves(p, launch_waves(p, t, b), st)) != TTM_OK) break;
                const BatchArgs a = make_args(p);
                if ((rc = launch_batched(p, a, X, A, B, C, Y, t, v, st)) != TTM_OK) break;   // warm-up
                double sum = 0.0;
                for (int r = 0; r < reps && rc == TTM_OK; ++r) {
                    if (hipMemsetAsync(flush, r & 0xff, flush_bytes, st) != hipSuccess ||
                        hipEventRecord(e0, st) != hipSuccess) { rc = TTM_ERR_HIP; break; }
                    if ((rc = launch_batched(p, a, X, A, B, C, Y, t, v, st)) != TTM_OK) break;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        rc = TTM_ERR_HIP;
                        break;
                    }
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = TTM_ERR_HIP; break; }
                    sum += ms;
                }
                if (rc) break;
                const double per = sum / reps;
                if (per < best) { best = per; bt = t; bb = b; bv = v; }
            }
        }
    }
    if (was_timing) ttm_timing_enable(1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(flush);
    if (rc == TTM_OK) rc = assign_waves(p, launch_waves(p, bt, bb), st);
    if (rc) return rc;
    p->threads = bt;
    p->blocks_per_cu = bb;
    p->variant = bv;
    if (p->exec) {   // the graph node keeps the old shape: rebuild on next use
        (void)hipGraphExecDestroy(p->exec);
        (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
    if (best_ms_out) *best_ms_out = best;
    if (!p->tune_cache.empty()) cache_store(p->tune_cache, p->tune_key, bt, bb, bv, best);
    return TTM_OK;
}

}  // extern "C"
