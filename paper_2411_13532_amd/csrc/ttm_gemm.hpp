// ttm_gemm.hpp -- a strided matrix-core GEMM used for the unfolded
// contractions of the adjoint:
//
//   Cout[b][m][n] (+)= sum_k opA(m, k) * opB(k, n)
//   opA(m, k) = A[b*sab + m*sam + ko*sako + ki*saki],   k = ko*Ki + ki
//   opB(k, n) = sum_{p < P} B[b*sbb + p*sbp + n*sbn + ko*sbko + ki*sbki]
//
// The two-level k index lets one call contract a pair of tensor modes whose
// strides do not merge (an unfolding read in place), and the optional sum over
// P partials folds a fixed-order reduction into the load.  Tiles of 64 x 64
// outputs, 4 waves each owning 32 x 32; both operands are staged through LDS
// in the k-contiguous fragment layout (one 16-byte LDS word per lane and
// k-group), whatever their strides in memory.  Split-K over grid.y writes
// per-split partials that a fixed-order reduction sums.
#pragma once
#include "ttm_device.hpp"

namespace ttm {

// K must be below 2^32 (the k split uses 32-bit division).
struct GemmArgs {
    const void *A, *B;
    void *C;
    int64_t M, N, K, Ki;
    int64_t sab, sam, sako, saki;
    int64_t sbb, sbn, sbko, sbki, sbp;
    int P;
    int64_t scb, scm, scn;
    int64_t k_per_split;   // k range of one grid.y split (multiple of the chunk)
    int64_t scs;           // stride between split partials in C
    int vec_a, vec_b;      // 1: the operand's unit-stride dimension can be read 16 bytes at a time
                           // (selects the kernel instantiation)
};

template <int MATH>
struct GemmCfg {
    typedef MathTraits<MATH> TR;
    typedef typename TR::lds_t LT;
    typedef typename TR::acc_t T;
    static constexpr int VE = TR::VE, KG = TR::KG;
    static constexpr int KT = 2 * KG;
    static constexpr int ROWB = KT * int(sizeof(LT)) + 16;
    static constexpr int TILEB = 64 * ROWB;
    static constexpr bool SPLIT = (MATH == M_BF16X3);
    static constexpr int PER = 64 * KT / 256;   // elements per thread per operand tile
};

// VA / VB: the operand's loads are 16-byte vectors (GemmArgs::vec_a / vec_b).
template <int MATH, bool VA, bool VB>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs a) {
    typedef GemmCfg<MATH> CF;
    typedef typename CF::T T;
    typedef typename CF::LT LT;
    typedef MathTraits<MATH> TR;
    typedef typename TR::accv_t accv_t;
    constexpr int KT = CF::KT, KG = CF::KG, PER = CF::PER;
    // [operand A|B][buffer 0|1][hi|lo]
    __shared__ __align__(16) unsigned char lds[2 * 2 * CF::TILEB * (CF::SPLIT ? 2 : 1)];
    auto tile = [&](int op, int buf, int lo) -> unsigned char * {
        return lds + ((op * 2 + buf) * (CF::SPLIT ? 2 : 1) + lo) * CF::TILEB;
    };

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = int64_t(blockIdx.x % ((a.M + 63) / 64)) * 64;
    const int64_t n0 = int64_t(blockIdx.x / ((a.M + 63) / 64)) * 64;
    const int64_t b = blockIdx.z;
    const int64_t kb = int64_t(blockIdx.y) * a.k_per_split;
    const int64_t ke = a.K < kb + a.k_per_split ? a.K : kb + a.k_per_split;
    const int64_t nch = ke > kb ? ceil_div(ke - kb, KT) : 0;
    const T *Ap = static_cast<const T *>(a.A) + b * a.sab;
    const T *Bp = static_cast<const T *>(a.B) + b * a.sbb;

    // Element e of a thread's share: along k when the operand is k-contiguous
    // (coalesced k runs), along m/n otherwise (coalesced m/n runs).
    const bool a_kfast = a.saki == 1;
    const bool b_kfast = a.sbki == 1;
    T pa[PER], pb[PER];
    auto coords = [&](bool kfast, int e, int &r, int &kk) {
        const int idx = tid + 256 * e;
        r = kfast ? idx / KT : idx % 64;
        kk = kfast ? idx % KT : idx / 64;
    };
    // Vector form of the same share: group e4 of VG consecutive elements along
    // the unit-stride dimension, read with one 16-byte load (flags set by the
    // host where strides, extents and alignment allow it); element u of group
    // e4 is element e4 * VG + u of the scalar share's numbering.
    constexpr int VG = 16 / int(sizeof(T));
    auto vcoords = [&](bool kfast, int e4, int &r, int &kk) {
        const int idx = tid + 256 * e4;
        r = kfast ? idx / (KT / VG) : (idx % (64 / VG)) * VG;
        kk = kfast ? (idx % (KT / VG)) * VG : idx / (64 / VG);
    };
    auto kdecomp = [&](int64_t k, int64_t &ko, int64_t &ki) {
        ko = int64_t(uint32_t(k) / uint32_t(a.Ki));
        ki = k - ko * a.Ki;
    };
    auto velem = [](const V16 &v, int u) -> T {
        if constexpr (sizeof(T) == 8) return v.d[u];
        else return v.f[u];
    };
    // Branch-free: out-of-range elements read element (0, 0) (always valid)
    // and are zeroed, so every load of a chunk is in flight at once.
    auto fetch = [&](int64_t ch) {
        const int64_t k0 = kb + ch * KT;
        if constexpr (VA) {
#pragma unroll
            for (int e4 = 0; e4 < PER / VG; ++e4) {
                int r, kk;
                vcoords(a_kfast, e4, r, kk);
                const int64_t m = m0 + r, k = k0 + kk;
                const bool ok = (a_kfast ? m < a.M : m + VG <= a.M) && (a_kfast ? k + VG <= ke : k < ke);
                int64_t ko, ki;
                kdecomp(k, ko, ki);
                const V16 v = ld16(Ap + (ok ? m * a.sam + ko * a.sako + ki * a.saki : 0));
#pragma unroll
                for (int u = 0; u < VG; ++u) pa[e4 * VG + u] = ok ? velem(v, u) : T(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                int r, kk;
                coords(a_kfast, e, r, kk);
                const int64_t m = m0 + r, k = k0 + kk;
                const bool ok = m < a.M && k < ke;
                int64_t ko, ki;
                kdecomp(k, ko, ki);
                const T v = Ap[ok ? m * a.sam + ko * a.sako + ki * a.saki : 0];
                pa[e] = ok ? v : T(0);
            }
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) pb[e] = T(0);
        for (int p = 0; p < a.P; ++p) {
            if constexpr (VB) {
#pragma unroll
                for (int e4 = 0; e4 < PER / VG; ++e4) {
                    int r, kk;
                    vcoords(b_kfast, e4, r, kk);
                    const int64_t n = n0 + r, k = k0 + kk;
                    const bool ok = (b_kfast ? n < a.N : n + VG <= a.N) && (b_kfast ? k + VG <= ke : k < ke);
                    int64_t ko, ki;
                    kdecomp(k, ko, ki);
                    const V16 v = ld16(Bp + (ok ? int64_t(p) * a.sbp + n * a.sbn + ko * a.sbko + ki * a.sbki : 0));
#pragma unroll
                    for (int u = 0; u < VG; ++u) pb[e4 * VG + u] += ok ? velem(v, u) : T(0);
                }
            } else {
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    int r, kk;
                    coords(b_kfast, e, r, kk);
                    const int64_t n = n0 + r, k = k0 + kk;
                    const bool ok = n < a.N && k < ke;
                    int64_t ko, ki;
                    kdecomp(k, ko, ki);
                    const T v = Bp[ok ? int64_t(p) * a.sbp + n * a.sbn + ko * a.sbko + ki * a.sbki : 0];
                    pb[e] += ok ? v : T(0);
                }
            }
        }
    };
    auto put = [&](unsigned char *hi, unsigned char *lo, int r, int kk, T v) {
        const int off = r * CF::ROWB + kk * int(sizeof(LT));
        if constexpr (MATH == M_BF16 || MATH == M_BF16X3) {
            uint32_t h, l;
            bf16_split(v, h, l);
            *reinterpret_cast<uint16_t *>(hi + off) = uint16_t(h);
            if constexpr (CF::SPLIT) *reinterpret_cast<uint16_t *>(lo + off) = uint16_t(l);
        } else {
            *reinterpret_cast<T *>(hi + off) = v;
        }
    };
    // element e of a share sits at (r, kk) of the scalar or of the vector numbering
    auto ecoords = [&](bool vec, bool kfast, int e, int &r, int &kk) {
        if (vec) {
            vcoords(kfast, e / VG, r, kk);
            const int du = e % VG;
            kk += kfast ? du : 0;
            r += kfast ? 0 : du;
        } else {
            coords(kfast, e, r, kk);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int r, kk;
            ecoords(VA, a_kfast, e, r, kk);
            put(tile(0, buf, 0), CF::SPLIT ? tile(0, buf, 1) : nullptr, r, kk, pa[e]);
            ecoords(VB, b_kfast, e, r, kk);
            put(tile(1, buf, 0), CF::SPLIT ? tile(1, buf, 1) : nullptr, r, kk, pb[e]);
        }
    };

    accv_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = zero_accv<accv_t>();

    if (nch > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();
    for (int64_t ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) fetch(ch + 1);
        const int buf = int(ch & 1);
#pragma unroll
        for (int kg = 0; kg < 2; ++kg) {
            V16 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int ra = (wm * 32 + i * 16 + l16) * CF::ROWB + kg * 64 + g * 16;
                const int rb = (wn * 32 + i * 16 + l16) * CF::ROWB + kg * 64 + g * 16;
                ah[i].u = *reinterpret_cast<const u32x4 *>(tile(0, buf, 0) + ra);
                bh[i].u = *reinterpret_cast<const u32x4 *>(tile(1, buf, 0) + rb);
                if constexpr (CF::SPLIT) {
                    al[i].u = *reinterpret_cast<const u32x4 *>(tile(0, buf, 1) + ra);
                    bl[i].u = *reinterpret_cast<const u32x4 *>(tile(1, buf, 1) + rb);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    mma_kgroup<MATH == M_BF16X3 ? M_BF16 : MATH>(acc[i][j], ah[i], bh[j]);
                    if constexpr (CF::SPLIT) {
                        mma_kgroup<M_BF16>(acc[i][j], ah[i], bl[j]);
                        mma_kgroup<M_BF16>(acc[i][j], al[i], bh[j]);
                    }
                }
        }
        if (ch + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }

    T *Cp = static_cast<T *>(a.C) + b * a.scb + int64_t(blockIdx.y) * a.scs;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 32 + i * 16 + TR::acc_row(g, r);
                const int64_t n = n0 + wn * 32 + j * 16 + l16;
                if (m < a.M && n < a.N) Cp[m * a.scm + n * a.scn] = acc[i][j][r];
            }
}

// out[e] = sum_{s < S} part[s * stride + e], increasing s.
template <typename T>
__global__ void __launch_bounds__(256) k_sum_splits(const T *part, int64_t stride, int S, int64_t n, T *out) {
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        T s = T(0);
        int k = 0;
        for (; k + 4 <= S; k += 4) {   // four loads in flight, summed in order
            const T v0 = part[k * stride + e], v1 = part[(k + 1) * stride + e];
            const T v2 = part[(k + 2) * stride + e], v3 = part[(k + 3) * stride + e];
            s += v0; s += v1; s += v2; s += v3;
        }
        for (; k < S; ++k) s += part[k * stride + e];
        out[e] = s;
    }
}

}  // namespace ttm
