// ttm_chain.hip -- Y = X x1 A x2 B x3 C on one MI355X (gfx950).
//
// Three kernels per call:
//   1. k_prep_factors : copy A, B, C into the workspace in the operand format
//      of the chosen arithmetic (double, float, or bfloat16 hi/lo), with rows
//      and columns zero-padded to the tile grid so no later load needs a guard.
//   2. k_slab : one workgroup per (i1, i2-range).  It streams its rows of X
//      once from HBM through an LDS double buffer and contracts mode 3 on the
//      matrix cores, W = X[i1, rows, :] C^T.  The W tile never leaves the
//      registers: its accumulator layout is reused directly as the k-major
//      operand of the mode-2 contraction V[i1] += B[:, rows] W, which also
//      stays in registers.  At the end the workgroup writes its partial
//      V[i1] (J2 x J3, float) -- the only intermediate that reaches HBM
//      (1/I3 of X's element count times J2*J3/I2, a few percent of X's bytes).
//   3. k_mode1 : Y = A V_(1), summing the partials of V in a fixed order
//      (no atomics, so every call is bitwise reproducible).
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <utility>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

constexpr int SLAB_TM = 128;     // rows of X[i1] per tile
constexpr int SLAB_THREADS = 256;

struct PrepArgs {
    const void *src[3];
    void *hi[3];
    void *lo[3];
    int64_t J[3], I[3], Jpad[3], ld[3];
    int perm32[3];   // 1: store columns in the mode-2 operand order (see below)
};

// Column position of source column c in a mode-2 bf16 operand row.  Inside
// every aligned block of 32 columns, accumulator rows 4g..4g+3 of the first
// 16-row block and 4g..4g+3 of the second one are the 8 k values of lane
// group g (slab_mode2); storing them next to each other lets one 16-byte
// load fetch the whole fragment.
__host__ __device__ inline int64_t mode2_col(int64_t c) {
    const int64_t q = c & 31, base = c - q;
    return q < 16 ? base + 8 * (q >> 2) + (q & 3) : base + 8 * ((q - 16) >> 2) + 4 + (q & 3);
}

// Factor n of shape J x I (row-major, float or double) -> padded Jpad x ld
// operand array(s).  For bfloat16 operands `hi` gets rne(v) and `lo` (when
// non-null) gets rne(v - hi).
template <typename ST, int MATH>
__global__ void __launch_bounds__(256) k_prep_factors(PrepArgs a) {
    const int f = blockIdx.y;
    const int64_t n = a.Jpad[f] * a.ld[f];
    const ST *src = static_cast<const ST *>(a.src[f]);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = e / a.ld[f], c = e % a.ld[f];
        const bool in = r < a.J[f] && c < a.I[f];
        if constexpr (MATH == M_BF16 || MATH == M_BF16X3) {
            const float v = in ? float(src[r * a.I[f] + c]) : 0.f;
            uint32_t h, l;
            bf16_split(v, h, l);
            const int64_t dst = a.perm32[f] ? r * a.ld[f] + mode2_col(c) : e;
            static_cast<uint16_t *>(a.hi[f])[dst] = uint16_t(h);
            if (a.lo[f]) static_cast<uint16_t *>(a.lo[f])[dst] = uint16_t(l);
        } else {
            typedef typename MathTraits<MATH>::fac_t FT;
            static_cast<FT *>(a.hi[f])[e] = in ? FT(src[r * a.I[f] + c]) : FT(0);
        }
    }
}

struct SlabArgs {
    const void *X;
    int64_t I1, I2, I3;
    const void *Chi, *Clo;  // [J3pad][ldc]
    int64_t ldc;
    const void *Bhi, *Blo;  // [J2pad][ldb]
    int64_t ldb;
    void *V;                // [I1][P][J2pad][J3pad]
    int64_t J2pad, J3pad;
    int P, S;
    int64_t rows_per_split;
    int x_vec;              // 1: rows of X are 16-byte aligned and I3 is a multiple of the vector width
};

// ---------------------------------------------------------------------------
// Loading one 16-byte LDS operand group (VE values of the operand type LT)
// from X of storage type XT.  `raw` keeps what was fetched until it is
// converted and stored after the current chunk's matrix-core work.
// ---------------------------------------------------------------------------
template <typename XT, typename LT> struct XGroup;

template <typename T> struct XGroup<T, T> {          // same type: one 16-byte load
    static constexpr int VE = 16 / sizeof(T);
    V16 raw;
    // row: this group's row of X; ok: row and k in range; safe: any valid address
    __device__ void fetch(const T *row, int64_t k, int64_t I3, bool ok, bool vec, const T *safe) {
        if (vec) {
            raw = ld16(ok ? row + k : safe);
            if (!ok) raw = zero16();
            return;
        }
        T tmp[VE];
#pragma unroll
        for (int e = 0; e < VE; ++e) tmp[e] = (ok && k + e < I3) ? row[k + e] : T(0);
        __builtin_memcpy(&raw, tmp, 16);
    }
    __device__ void store(unsigned char *hi, unsigned char *) const { *reinterpret_cast<u32x4 *>(hi) = raw.u; }
};

template <> struct XGroup<uint16_t, float> {        // bf16 X, float operands: 8-byte load
    static constexpr int VE = 4;
    u32x2 raw;
    __device__ void fetch(const uint16_t *row, int64_t k, int64_t I3, bool ok, bool vec, const uint16_t *safe) {
        if (vec) {
            raw = *reinterpret_cast<const u32x2 *>(ok ? row + k : safe);
            if (!ok) raw = u32x2{0u, 0u};
            return;
        }
        uint32_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = (ok && k + e < I3) ? row[k + e] : 0u;
        raw = u32x2{pack2(h[0], h[1]), pack2(h[2], h[3])};
    }
    __device__ void store(unsigned char *hi, unsigned char *) const {
        f32x4 v;
        v[0] = __uint_as_float(raw[0] << 16);
        v[1] = __uint_as_float(raw[0] & 0xffff0000u);
        v[2] = __uint_as_float(raw[1] << 16);
        v[3] = __uint_as_float(raw[1] & 0xffff0000u);
        *reinterpret_cast<f32x4 *>(hi) = v;
    }
};

template <> struct XGroup<float, uint16_t> {        // float X, bf16 operands: 32-byte load, split on store
    static constexpr int VE = 8;
    V16 raw0, raw1;
    __device__ void fetch(const float *row, int64_t k, int64_t I3, bool ok, bool vec, const float *safe) {
        if (vec) {
            const float *p = ok ? row + k : safe;
            raw0 = ld16(p);
            raw1 = ld16(p + 4);
            if (!ok) { raw0 = zero16(); raw1 = zero16(); }
            return;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            raw0.f[e] = (ok && k + e < I3) ? row[k + e] : 0.f;
            raw1.f[e] = (ok && k + 4 + e < I3) ? row[k + 4 + e] : 0.f;
        }
    }
    __device__ void store(unsigned char *hi, unsigned char *lo) const {
        const float v[8] = {raw0.f[0], raw0.f[1], raw0.f[2], raw0.f[3], raw1.f[0], raw1.f[1], raw1.f[2], raw1.f[3]};
        u32x4 h, l;
        bf16_split8(v, h, lo ? &l : nullptr);
        *reinterpret_cast<u32x4 *>(hi) = h;
        if (lo) *reinterpret_cast<u32x4 *>(lo) = l;
    }
};

template <int MATH, typename XT> struct SlabCfg {
    typedef MathTraits<MATH> TR;
    typedef typename TR::lds_t LT;
    static constexpr int VE = TR::VE;
    static constexpr int KG = TR::KG;             // k per k-group (64 bytes of LT per row)
    static constexpr int KC = 2 * KG;             // k per chunk (128 bytes of LT per row)
    static constexpr int ROWB = KC * int(sizeof(LT)) + 16;   // padded LDS row stride
    static constexpr int TILEB = SLAB_TM * ROWB;
    static constexpr bool XLO = (MATH == M_BF16X3) && std::is_same<XT, float>::value;
    static constexpr int GROUPS = SLAB_TM * 8 / SLAB_THREADS;  // 16-byte LDS groups per thread per chunk
    static constexpr size_t lds_bytes() { return size_t(TILEB) * 2 * (XLO ? 2 : 1); }
};

// Mode-2 step: V[jb][nb] += B[j2 rows, tile rows] * W[tile rows, cols].
// f32/f64: per 16-row block, the accumulator register r of lane (g, c) is
// W[acc_row(g, r)][c], so MFMA r takes k-slot g <-> row acc_row(g, r).
template <int MATH, int MB, int NBW, int JB>
__device__ __forceinline__ void slab_mode2(typename MathTraits<MATH>::accv_t (&vacc)[JB][NBW],
                                           const typename MathTraits<MATH>::accv_t (&wacc)[MB][NBW],
                                           const SlabArgs &a, int jbase, int64_t wrow0, int l16, int g) {
    if constexpr (MATH == M_F32 || MATH == M_F64) {
        typedef typename MathTraits<MATH>::fac_t FT;
        const FT *Bp = static_cast<const FT *>(a.Bhi);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                {
                    const FT *brow = Bp + int64_t((jbase + jb) * 16 + l16) * a.ldb + wrow0 + mb * 16;
                    FT bv[4];
                    if constexpr (MATH == M_F32) {
                        V16 t = ld16(brow + 4 * g);        // rows 4g .. 4g+3
#pragma unroll
                        for (int r = 0; r < 4; ++r) bv[r] = t.f[r];
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) bv[r] = brow[MathTraits<MATH>::acc_row(g, r)];
                    }
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if constexpr (MATH == M_F32) vacc[jb][nb] = mfma_f32(bv[r], wacc[mb][nb][r], vacc[jb][nb]);
                            else vacc[jb][nb] = mfma_f64(bv[r], wacc[mb][nb][r], vacc[jb][nb]);
                        }
                }
            }
            // keep the next block's loads from being hoisted (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        // bf16: two stacked 16-row blocks give a lane the 8 values
        // {W[32p + 4g + e], W[32p + 16 + 4g + e]}, e = 0..3 -> one k-slot group;
        // the B operand stores those 8 columns contiguously (mode2_col).
        const uint16_t *Bh = static_cast<const uint16_t *>(a.Bhi);
        const uint16_t *Bl = static_cast<const uint16_t *>(a.Blo);
#pragma unroll
        for (int p = 0; p < MB / 2; ++p) {
            u32x4 wh[NBW], wl[NBW];
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const float v[8] = {wacc[2 * p][nb][0], wacc[2 * p][nb][1], wacc[2 * p][nb][2], wacc[2 * p][nb][3],
                                    wacc[2 * p + 1][nb][0], wacc[2 * p + 1][nb][1], wacc[2 * p + 1][nb][2],
                                    wacc[2 * p + 1][nb][3]};
                if constexpr (MATH == M_BF16X3) bf16_split8(v, wh[nb], &wl[nb]);
                else wh[nb] = bf16_round8(v);
            }
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                const int64_t off = int64_t((jbase + jb) * 16 + l16) * a.ldb + wrow0 + 32 * p + 8 * g;
                const u32x4 bh = ld16(Bh + off).u;
                if constexpr (MATH == M_BF16X3) {
                    const u32x4 bl = ld16(Bl + off).u;
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) {
                        vacc[jb][nb] = mfma_bf16(bh, wh[nb], vacc[jb][nb]);
                        vacc[jb][nb] = mfma_bf16(bh, wl[nb], vacc[jb][nb]);
                        vacc[jb][nb] = mfma_bf16(bl, wh[nb], vacc[jb][nb]);
                    }
                } else {
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) vacc[jb][nb] = mfma_bf16(bh, wh[nb], vacc[jb][nb]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// One workgroup: 4 waves arranged WR x WC over (tile rows) x (columns j3).
// Wave (wr, wc) owns RW = 128 / WR rows of every 128-row tile and NBW 16-wide
// column blocks.  The workgroup covers columns blockIdx.y * (WC*NBW*16) ...
// and j2 blocks blockIdx.z * JBMAX ...; its partial index of V is s*WR + wr.
template <int MATH, typename XT, int WC, int NBW, int JB>
__global__ void __launch_bounds__(SLAB_THREADS, 2) k_slab(const SlabArgs a) {
    typedef SlabCfg<MATH, XT> CF;
    typedef typename CF::LT LT;
    typedef typename MathTraits<MATH>::accv_t accv_t;
    typedef typename MathTraits<MATH>::acc_t acc_t;
    typedef typename MathTraits<MATH>::fac_t FT;
    constexpr int WR = 4 / WC, RW = SLAB_TM / WR, MB = RW / 16;
    constexpr int KG = CF::KG, KC = CF::KC, VE = CF::VE;
    constexpr int GROUPS = CF::GROUPS;
    static_assert(MB >= 2 && MB % 2 == 0, "row blocks per wave");

    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *tile_hi = smem;
    unsigned char *tile_lo = smem + 2 * CF::TILEB;   // used only when CF::XLO

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WC, wc = wave % WC;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t i1 = blockIdx.x / a.S;
    const int s = int(blockIdx.x % a.S);
    const int64_t row_begin = int64_t(s) * a.rows_per_split;
    const int64_t row_end = a.I2 < row_begin + a.rows_per_split ? a.I2 : row_begin + a.rows_per_split;
    const int64_t nrows = row_end > row_begin ? row_end - row_begin : 0;
    const int64_t col0 = int64_t(blockIdx.y) * (WC * NBW * 16) + wc * NBW * 16;
    const int jbase = int(blockIdx.z) * JB;

    const XT *Xs = static_cast<const XT *>(a.X) + i1 * a.I2 * a.I3;
    const int64_t nk = ceil_div(a.I3, KC);
    const int64_t ntiles = ceil_div(nrows, SLAB_TM);
    const int64_t nq = ntiles * nk;
    const bool vec = a.x_vec != 0;

    accv_t vacc[JB][NBW];
    accv_t wacc[MB][NBW];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) vacc[jb][nb] = zero_accv<accv_t>();

    XGroup<XT, LT> pre[GROUPS];
    auto fetch = [&](int64_t t, int64_t kc) {
        const int64_t r0 = row_begin + t * SLAB_TM;
#pragma unroll
        for (int j = 0; j < GROUPS; ++j) {
            const int gi = tid + SLAB_THREADS * j;
            const int r = gi >> 3, cg = gi & 7;
            const int64_t grow = r0 + r;
            const int64_t k = kc * KC + cg * VE;
            pre[j].fetch(Xs + grow * a.I3, k, a.I3, grow < row_end && k < a.I3, vec, Xs);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < GROUPS; ++j) {
            const int gi = tid + SLAB_THREADS * j;
            const int r = gi >> 3, cg = gi & 7;
            const int off = buf * CF::TILEB + r * CF::ROWB + cg * 16;
            pre[j].store(tile_hi + off, CF::XLO ? tile_lo + off : nullptr);
        }
    };
    const FT *Ch = static_cast<const FT *>(a.Chi);
    const FT *Cl = static_cast<const FT *>(a.Clo);

    if (nq > 0) {
        fetch(0, 0);
        store(0);
    }
    __syncthreads();

    int64_t q = 0;
    int64_t ft = 0, fkc = 1;   // chunk fetched next (tile, k chunk)
    if (fkc == nk) { fkc = 0; ft = 1; }
    for (int64_t t = 0; t < ntiles; ++t) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) wacc[mb][nb] = zero_accv<accv_t>();

        for (int64_t kc = 0; kc < nk; ++kc, ++q) {
            const bool more = q + 1 < nq;
            if (more) fetch(ft, fkc);

            const int buf = int(q & 1);
#pragma unroll
            for (int kg = 0; kg < 2; ++kg) {
                const int64_t k0 = kc * KC + kg * KG + g * VE;
                V16 bh[NBW], bl[NBW];
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    const int64_t off = (col0 + nb * 16 + l16) * a.ldc + k0;
                    bh[nb] = ld16(Ch + off);
                    if constexpr (MATH == M_BF16X3) bl[nb] = ld16(Cl + off);
                }
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int loff = buf * CF::TILEB + (wr * RW + mb * 16 + l16) * CF::ROWB + kg * 64 + g * 16;
                    V16 ah;
                    ah.u = *reinterpret_cast<const u32x4 *>(tile_hi + loff);
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) {
                        mma_kgroup<MATH == M_BF16X3 ? M_BF16 : MATH>(wacc[mb][nb], ah, bh[nb]);
                        if constexpr (MATH == M_BF16X3) mma_kgroup<M_BF16>(wacc[mb][nb], ah, bl[nb]);
                    }
                    if constexpr (CF::XLO) {
                        V16 al;
                        al.u = *reinterpret_cast<const u32x4 *>(tile_lo + loff);
#pragma unroll
                        for (int nb = 0; nb < NBW; ++nb) mma_kgroup<M_BF16>(wacc[mb][nb], al, bh[nb]);
                    }
                }
            }
            if (more) {
                store(buf ^ 1);
                if (++fkc == nk) { fkc = 0; ++ft; }
            }
            __syncthreads();
        }
        const int64_t wrow0 = row_begin + t * SLAB_TM + wr * RW;
        slab_mode2<MATH, MB, NBW, JB>(vacc, wacc, a, jbase, wrow0, l16, g);
    }

    // Partial V[i1][s*WR + wr][j2][j3]: lane (g, c) register r holds
    // row j2 = 16*jb + acc_row(g, r), column j3 = col0 + 16*nb + c.
    acc_t *V = static_cast<acc_t *>(a.V);
    const int64_t part = int64_t(s) * WR + wr;
    acc_t *Vp = V + (i1 * a.P + part) * a.J2pad * a.J3pad;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j2 = int64_t(jbase + jb) * 16 + MathTraits<MATH>::acc_row(g, r);
                Vp[j2 * a.J3pad + col0 + nb * 16 + l16] = vacc[jb][nb][r];
            }
}

// ---------------------------------------------------------------------------
// k_slab_dma: the same computation as k_slab for the common case where X is
// already in the operand format (bf16 X with bf16/bf16x3 arithmetic, f32 X
// with f32, f64 X with f64), rows are 16-byte aligned and I3 is a multiple of
// the 256-byte chunk.  X goes from HBM straight into LDS (global_load_lds,
// no register staging) in chunks of 128 rows x 256 bytes, double-buffered in
// two LDS arrays so that the compiler's wait before each barrier covers
// exactly the chunk about to be used.  Inside a chunk the 16-byte words of a
// row are XOR-swizzled by (row & 15): a 16-byte LDS read is served 16 lanes
// at a time over 64 banks (256 bytes), and the 16 rows of an operand
// fragment then land on 16 distinct 16-byte bank groups.  Chunks are 256
// bytes per row (64 KiB of LDS, two workgroups per compute unit).  Rows past
// the end of a slab range are read from a clamped (valid) row and their W
// rows zeroed before the mode-2 step.
// ---------------------------------------------------------------------------
template <int MATH, int WC, int NBW, int JB>
__global__ void __launch_bounds__(SLAB_THREADS, 2) k_slab_dma(const SlabArgs a) {
    typedef MathTraits<MATH> TR;
    typedef typename TR::lds_t LT;
    typedef typename TR::accv_t accv_t;
    typedef typename TR::acc_t acc_t;
    typedef typename TR::fac_t FT;
    constexpr int WR = 4 / WC, RW = SLAB_TM / WR, MB = RW / 16;
    constexpr int VE = TR::VE, KG = TR::KG;
    constexpr int ROWB = 256;                           // bytes of a row per chunk
    constexpr int KC = ROWB / int(sizeof(LT));         // k per chunk
    constexpr int NKG = ROWB / 64;                      // k-groups per chunk
    constexpr int STAGE = SLAB_TM * ROWB;
    constexpr int WPR = ROWB / 16;                      // 16-byte words per row
    constexpr int RPI = 1024 / ROWB;                    // rows per wave instruction
    constexpr int NDMA = SLAB_TM / 4 / RPI;             // instructions per wave per stage
    static_assert(MB >= 2 && MB % 2 == 0, "row blocks per wave");

    __shared__ __align__(1024) unsigned char st0[STAGE];
    __shared__ __align__(1024) unsigned char st1[STAGE];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WC, wc = wave % WC;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t i1 = blockIdx.x / a.S;
    const int s = int(blockIdx.x % a.S);
    const int64_t row_begin = int64_t(s) * a.rows_per_split;
    const int64_t row_end = a.I2 < row_begin + a.rows_per_split ? a.I2 : row_begin + a.rows_per_split;
    const int64_t nrows = row_end > row_begin ? row_end - row_begin : 0;
    const int64_t col0 = int64_t(blockIdx.y) * (WC * NBW * 16) + wc * NBW * 16;
    const int jbase = int(blockIdx.z) * JB;

    const LT *Xs = static_cast<const LT *>(a.X) + i1 * a.I2 * a.I3;
    const int64_t nk = a.I3 / KC;
    const int64_t ntiles = ceil_div(nrows, SLAB_TM);
    const int64_t nq = ntiles * nk;
    const FT *Ch = static_cast<const FT *>(a.Chi);
    const FT *Cl = static_cast<const FT *>(a.Clo);

    // DMA of chunk (t, kc) into one stage: wave w moves rows 32w .. 32w+31,
    // RPI rows per instruction; lane l fills slot (row, word l % WPR), which
    // holds logical word (l % WPR) ^ (row & 15) of that row.
    const int drow_in = lane / WPR, dpos = lane % WPR;
    auto dma = [&](unsigned char *stage, int64_t t, int64_t kc) {
        const int64_t r0 = row_begin + t * SLAB_TM;
#pragma unroll
        for (int j = 0; j < NDMA; ++j) {
            const int row = wave * 32 + RPI * j + drow_in;
            int64_t grow = r0 + row;
            grow = grow < row_end ? grow : row_end - 1;
            const int word = dpos ^ (row & 15);
            const LT *src = Xs + grow * a.I3 + kc * KC + word * VE;
            dma16_to_lds(src, stage + (wave * 32 + RPI * j) * ROWB);
        }
    };

    accv_t vacc[JB][NBW];
    accv_t wacc[MB][NBW];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) vacc[jb][nb] = zero_accv<accv_t>();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) wacc[mb][nb] = zero_accv<accv_t>();

    // one chunk of matrix-core work from a stage; the factor fragments of the
    // next k-group are loaded while the current one is on the matrix cores
    auto compute = [&](const unsigned char *stage, int64_t kc) {
        V16 bh[2][NBW], bl[2][NBW];
        auto load_c = [&](int slot, int kg) {
            const int64_t k0 = kc * KC + kg * KG + g * VE;
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int64_t off = (col0 + nb * 16 + l16) * a.ldc + k0;
                bh[slot][nb] = ld16(Ch + off);
                if constexpr (MATH == M_BF16X3) bl[slot][nb] = ld16(Cl + off);
            }
        };
        load_c(0, 0);
#pragma unroll
        for (int kg = 0; kg < NKG; ++kg) {
            if (kg + 1 < NKG) load_c((kg + 1) & 1, kg + 1);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int row = wr * RW + mb * 16 + l16;
                const int word = (kg * 4 + g) ^ (row & 15);
                V16 ah;
                ah.u = *reinterpret_cast<const u32x4 *>(stage + row * ROWB + word * 16);
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    mma_kgroup<MATH == M_BF16X3 ? M_BF16 : MATH>(wacc[mb][nb], ah, bh[kg & 1][nb]);
                    if constexpr (MATH == M_BF16X3) mma_kgroup<M_BF16>(wacc[mb][nb], ah, bl[kg & 1][nb]);
                }
            }
        }
    };
    // end of a 128-row tile: zero rows past the range, mode-2 step, reset W
    auto tile_end = [&](int64_t t) {
        const int64_t wrow0 = row_begin + t * SLAB_TM + wr * RW;
        if (row_begin + (t + 1) * SLAB_TM > row_end) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool dead = wrow0 + mb * 16 + TR::acc_row(g, r) >= row_end;
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb)
                        if (dead) wacc[mb][nb][r] = acc_t(0);
                }
        }
        slab_mode2<MATH, MB, NBW, JB>(vacc, wacc, a, jbase, wrow0, l16, g);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) wacc[mb][nb] = zero_accv<accv_t>();
    };

    int64_t t = 0, kc = 0;       // chunk being computed
    int64_t ft = 0, fkc = 0;     // chunk fetched next
    auto next = [&](int64_t &tt, int64_t &kk) { if (++kk == nk) { kk = 0; ++tt; } };
    if (nq > 0) {
        dma(st0, ft, fkc);
        next(ft, fkc);
    }
    for (int64_t q = 0; q < nq; q += 2) {
        __syncthreads();                       // chunk q is in st0; st1 is free
        if (q + 1 < nq) { dma(st1, ft, fkc); next(ft, fkc); }
        compute(st0, kc);
        if (kc == nk - 1) tile_end(t);
        next(t, kc);
        if (q + 1 >= nq) break;
        __syncthreads();                       // chunk q+1 is in st1; st0 is free
        if (q + 2 < nq) { dma(st0, ft, fkc); next(ft, fkc); }
        compute(st1, kc);
        if (kc == nk - 1) tile_end(t);
        next(t, kc);
    }

    acc_t *Vp = static_cast<acc_t *>(a.V) + (i1 * a.P + int64_t(s) * WR + wr) * a.J2pad * a.J3pad;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j2 = int64_t(jbase + jb) * 16 + TR::acc_row(g, r);
                Vp[j2 * a.J3pad + col0 + nb * 16 + l16] = vacc[jb][nb][r];
            }
}

// s_waitcnt with only the vector-memory count limited (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt and lgkmcnt at their maxima).

// Mode-2 step for the bf16 forms with the B loads software-pipelined: W is
// first converted to its bf16 operand pairs (freeing the accumulators), then
// the tile's B fragments are taken in rounds of four 16-row blocks of j2 (hi
// and lo) over 32 rows, and the loads of round r + 1 are issued before the
// products of round r, so each round waits for loads that have had a round of
// products to land instead of a full L2 round trip.
template <int MATH, int MB, int NBW, int JB>
__device__ __forceinline__ void slab_mode2_pipe(typename MathTraits<MATH>::accv_t (&vacc)[JB][NBW],
                                                typename MathTraits<MATH>::accv_t (&wacc)[MB][NBW],
                                                const SlabArgs &a, int jbase, int64_t wrow0, int l16, int g) {
    static_assert(MATH == M_BF16 || MATH == M_BF16X3, "bf16 forms");
    constexpr bool X3 = MATH == M_BF16X3;
    constexpr int JG = JB < 4 ? JB : 4, NG = JB / JG, R = (MB / 2) * NG;
    const uint16_t *Bh = static_cast<const uint16_t *>(a.Bhi);
    const uint16_t *Bl = static_cast<const uint16_t *>(a.Blo);
    u32x4 wh[MB / 2][NBW], wl[MB / 2][NBW];
#pragma unroll
    for (int p = 0; p < MB / 2; ++p)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) {
            const float v[8] = {wacc[2 * p][nb][0], wacc[2 * p][nb][1], wacc[2 * p][nb][2], wacc[2 * p][nb][3],
                                wacc[2 * p + 1][nb][0], wacc[2 * p + 1][nb][1], wacc[2 * p + 1][nb][2],
                                wacc[2 * p + 1][nb][3]};
            if constexpr (X3) bf16_split8(v, wh[p][nb], &wl[p][nb]);
            else wh[p][nb] = bf16_round8(v);
        }
    u32x4 bh[2][JG], bl[2][JG];
    auto load = [&](int r, int buf) __attribute__((always_inline)) {
        const int p = r / NG, j0 = (r % NG) * JG;
#pragma unroll
        for (int jj = 0; jj < JG; ++jj) {
            const int64_t off = int64_t((jbase + j0 + jj) * 16 + l16) * a.ldb + wrow0 + 32 * p + 8 * g;
            bh[buf][jj] = ld16(Bh + off).u;
            if constexpr (X3) bl[buf][jj] = ld16(Bl + off).u;
        }
    };
    load(0, 0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r + 1 < R) load(r + 1, (r + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
        const int p = r / NG, j0 = (r % NG) * JG, cb = r & 1;
#pragma unroll
        for (int jj = 0; jj < JG; ++jj)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                auto &acc = vacc[j0 + jj][nb];
                acc = mfma_bf16(bh[cb][jj], wh[p][nb], acc);
                if constexpr (X3) {
                    acc = mfma_bf16(bh[cb][jj], wl[p][nb], acc);
                    acc = mfma_bf16(bl[cb][jj], wh[p][nb], acc);
                }
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// k_slab_lc: the slab kernel with the factor C staged through LDS, for bf16 X
// with the bf16 and bf16x3 forms where four waves share the columns (WC == 4).
//
// In the register-fed kernels every wave loads its own C fragments from L2
// for every k-group of every 128-row tile: twice the bytes of X, and each of
// those loads sits in the same in-order vector-memory queue as the X copies,
// so its wait can include a copy.  Here one workgroup per compute unit runs
// eight waves over 256-row tiles: the C chunk of the workgroup's columns (hi
// and lo) is copied into LDS by the same direct-to-LDS copies as X, once per
// workgroup and chunk, halving the C traffic, and the matrix-core waves read
// both operands from LDS.  Wave (wr, wc) owns rows 128 wr .. 128 wr + 127 of
// each tile and NBW column blocks.
//
// Chunks are 128 bytes of each row (64 values).  X has three LDS stages (two
// chunks in flight), C two (one chunk ahead: it comes from L2).  Copies are
// issued C(q+1) then X(q+2), so before the barrier of chunk q a wave waits
// until at most its copies of X(q+1) are outstanding (explicit vmcnt).  The
// stage reads are ds_read_b128 issued through inline assembly, waited for
// with explicit lgkmcnt waits that the fragments depend on: the compiler
// therefore never adds a wait of its own for the copies in flight, which it
// cannot tell apart by stage.  The 16-byte words of a 128-byte row are XOR-
// swizzled by (row >> 1) & 7: the 16 rows of a fragment read cover all 64
// banks.  At the end of a tile the mode-2 step copies B once per workgroup
// into the tile's consumed X and C stages (mode2_lds below) for all eight
// waves to read.  The two row halves' V partials are added through LDS at
// the end.
// ---------------------------------------------------------------------------
constexpr int LC_THREADS = 512;
constexpr int LC_TM = 256;
constexpr int LC_XSTAGE = LC_TM * 128;               // 32 KiB

template <int OFF>
__device__ __forceinline__ u32x4 lds_read16_at(uint32_t addr) {
    static_assert(OFF >= 0 && OFF < 65536 && OFF % 16 == 0, "ds_read_b128 immediate offset");
    u32x4 v;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF) : "memory");
    return v;
}
// wait until at most N LDS reads of this wave are in flight
template <int N>
__device__ __forceinline__ void lds_wait() {
    static_assert(N >= 0 && N < 16, "lgkmcnt range");
    asm volatile("s_waitcnt lgkmcnt(%0)" : : "n"(N));
}
// makes r's value available only after the preceding wait (r was written by
// an LDS read issued through inline assembly)
__device__ __forceinline__ void lds_dep(u32x4 &r) { asm volatile("" : "+v"(r)); }
// Read order and waits of one chunk of k_slab_lc: per k-group NC C reads then
// MB X reads; group g = (kg, mb) needs reads up to need(g); before group g the
// reads up to issued(g) have been issued, keeping at most 12 in flight past
// the last read known to have returned.
template <int NC_, int MB, int NKG>
struct LcReadSched {
    static constexpr int NC = NC_, PER_KG = NC_ + MB, NR = NKG * PER_KG;
    static constexpr int need(int g) { return (g / MB) * PER_KG + NC + g % MB; }
    static constexpr int issued(int g) {
        if (g < 0) return 0;
        const int done = g == 0 ? 0 : need(g - 1) + 1;
        return done + 12 < NR ? done + 12 : NR;
    }
};
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N - 1, in order
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

template <int MATH, int NBW, int JB>
__global__ void __launch_bounds__(LC_THREADS, 1) k_slab_lc(const SlabArgs a) {
    typedef MathTraits<MATH> TR;
    typedef typename TR::accv_t accv_t;
    constexpr bool X3 = MATH == M_BF16X3;
    static_assert(MATH == M_BF16 || MATH == M_BF16X3, "bf16 forms");
    constexpr int WC = 4, RW = 128, MB = 8;
    constexpr int KC = 64, NKG = 2;                   // bf16 values per chunk row, k-groups per chunk
    constexpr int COLS = WC * NBW * 16;               // columns of the workgroup
    constexpr int CPART = COLS * 128;                 // bytes of one C part (hi or lo) per stage
    constexpr int CSTAGE = CPART * (X3 ? 2 : 1);
    constexpr int XOPS = LC_XSTAGE / 1024 / 8;        // X copy instructions per wave per chunk (4)
    constexpr int COPS = CSTAGE / 1024 / 8;           // C copy instructions per wave per chunk
    constexpr int NCF = NKG * NBW * (X3 ? 2 : 1);     // C fragments per chunk

    __shared__ __align__(1024) unsigned char xbuf[3 * LC_XSTAGE];
    __shared__ __align__(1024) unsigned char cbuf[2 * CSTAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / WC, wc = wave % WC;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t i1 = blockIdx.x / a.S;
    const int s = int(blockIdx.x % a.S);
    const int64_t row_begin = int64_t(s) * a.rows_per_split;
    const int64_t row_end = a.I2 < row_begin + a.rows_per_split ? a.I2 : row_begin + a.rows_per_split;
    const int64_t nrows = row_end > row_begin ? row_end - row_begin : 0;
    const int64_t colb = int64_t(blockIdx.y) * COLS;  // first column of the workgroup
    const int jbase = int(blockIdx.z) * JB;
    const uint16_t *Xs = static_cast<const uint16_t *>(a.X) + i1 * a.I2 * a.I3;
    const uint16_t *Ch = static_cast<const uint16_t *>(a.Chi);
    const uint16_t *Cl = static_cast<const uint16_t *>(a.Clo);
    const int64_t nk = a.I3 / KC;
    const int64_t ntiles = ceil_div(nrows, LC_TM);
    const int64_t nq = ntiles * nk;

    // copies: 8 rows (or columns) of 128 bytes per instruction; lane l fills
    // word l % 8 of row l / 8 with logical word (l % 8) ^ ((row >> 1) & 7).
    // Addresses are a uniform base plus a 32-bit lane offset (the host
    // guarantees 256 rows of X, the columns of C and B each span less than 2 GiB);
    // X's lane offsets change only at a tile whose rows run past the range,
    // where rows are clamped to the last one.
    const int drow = lane >> 3, dpos = lane & 7;
    const int64_t xrow_bytes = a.I3 * 2, crow_bytes = a.ldc * 2;
    uint32_t xlo[XOPS], clo[COPS];
    const uint32_t xrow_b32 = uint32_t(xrow_bytes);
    auto set_x_offsets = [&](int64_t r0) __attribute__((always_inline)) {
        // last row of the range relative to the tile, at most LC_TM - 1
        const int64_t last64 = row_end - 1 - r0;
        const int last = __builtin_amdgcn_readfirstlane(int(last64 < LC_TM - 1 ? last64 : LC_TM - 1));
#pragma unroll
        for (int j = 0; j < XOPS; ++j) {
            const int row = (wave * XOPS + j) * 8 + drow;
            const uint32_t rr = uint32_t(row < last ? row : last);
            xlo[j] = rr * xrow_b32 + uint32_t((dpos ^ ((row >> 1) & 7)) << 4);
        }
    };
#pragma unroll
    for (int j = 0; j < COPS; ++j) {
        const int idx = wave * COPS + j;
        const int col = (idx % (COLS / 8)) * 8 + drow;
        clo[j] = uint32_t(col) * uint32_t(crow_bytes) + uint32_t((dpos ^ ((col >> 1) & 7)) << 4);
    }
    const char *xslab = reinterpret_cast<const char *>(Xs);
    const char *cbase[2] = {reinterpret_cast<const char *>(Ch + colb * a.ldc),
                            reinterpret_cast<const char *>((X3 ? Cl : Ch) + colb * a.ldc)};
    // stage arguments are LDS byte addresses
    auto copy_x = [&](uint32_t stage, int64_t t, int kc) __attribute__((always_inline)) {
        const char *base = xslab + (row_begin + t * LC_TM) * xrow_bytes + kc * 128;
#pragma unroll
        for (int j = 0; j < XOPS; ++j) dma16s_to_lds_m0(base, xlo[j], stage + uint32_t((wave * XOPS + j) * 8 * 128));
    };
    auto copy_c = [&](uint32_t stage, int kc) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < COPS; ++j) {
            const int idx = wave * COPS + j;
            const int part = idx / (COLS / 8);         // 0: hi, 1: lo
            const int col0 = (idx % (COLS / 8)) * 8;
            dma16s_to_lds_m0(cbase[part] + kc * 128, clo[j], stage + uint32_t(part * CPART + col0 * 128));
        }
    };

    accv_t vacc[JB][NBW];
    accv_t wacc[MB][NBW];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) vacc[jb][nb] = zero_accv<accv_t>();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) wacc[mb][nb] = zero_accv<accv_t>();

    // per-lane LDS byte offsets of the fragment words of k-group kg: the
    // swizzle key (row >> 1) & 7 of rows 16 m + l16 is (l16 >> 1) & 7 for
    // every 16-row block, so block m adds the immediate m * 2048
    uint32_t xl[NKG], cl[NKG];
#pragma unroll
    for (int kg = 0; kg < NKG; ++kg) {
        const uint32_t w = uint32_t(((kg * 4 + g) ^ ((l16 >> 1) & 7)) << 4);
        xl[kg] = uint32_t((wr * RW + l16) * 128) + w;
        cl[kg] = uint32_t((wc * NBW * 16 + l16) * 128) + w;
    }
    const uint32_t xlds = lds_offset(xbuf), clds = lds_offset(cbuf);

    // one chunk of matrix-core work, in groups (k-group kg, 16-row block mb).
    // The chunk's LDS reads are issued in the order the groups consume them
    // (per k-group: its C fragments, then the X fragments of blocks 0 .. MB-1)
    // with at most 12 in flight (the LDS counter counts to 15; 12 keeps the
    // fragments within the registers at two waves per SIMD), and each group
    // waits only until its own operands have returned (LDS reads of a wave
    // return in order): the first products start after a few reads instead of
    // after all of them.
    typedef LcReadSched<NCF / NKG, MB, NKG> SC;
    auto compute = [&](uint32_t xs, uint32_t cs, auto &&after_group) __attribute__((always_inline)) {
        u32x4 rd[SC::NR];
        const uint32_t xa[NKG] = {xs + xl[0], xs + xl[1]};
        const uint32_t ca[NKG] = {cs + cl[0], cs + cl[1]};
        auto issue = [&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value, kg = i / SC::PER_KG, w = i % SC::PER_KG;
            if constexpr (w < SC::NC) {
                constexpr int nb = w / (X3 ? 2 : 1), part = w % (X3 ? 2 : 1);
                rd[i] = lds_read16_at<part * CPART + nb * 2048>(ca[kg]);
            } else {
                rd[i] = lds_read16_at<(w - SC::NC) * 2048>(xa[kg]);
            }
        };
        static_for<NKG * MB>([&](auto G) __attribute__((always_inline)) {
            constexpr int g = decltype(G)::value, kg = g / MB, mb = g % MB;
            constexpr int i0 = SC::issued(g - 1), i1 = SC::issued(g);
            static_for<i1 - i0>([&](auto J) __attribute__((always_inline)) {
                issue(std::integral_constant<int, i0 + decltype(J)::value>{});
            });
            lds_wait<i1 - SC::need(g) - 1>();
            constexpr int cb = kg * SC::PER_KG, xr = cb + SC::NC + mb;
            lds_dep(rd[xr]);
            if constexpr (mb == 0)
                static_for<SC::NC>([&](auto C) __attribute__((always_inline)) { lds_dep(rd[cb + decltype(C)::value]); });
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                wacc[mb][nb] = mfma_bf16(rd[xr], rd[cb + nb * (X3 ? 2 : 1)], wacc[mb][nb]);
                if constexpr (X3) wacc[mb][nb] = mfma_bf16(rd[xr], rd[cb + nb * 2 + 1], wacc[mb][nb]);
            }
            after_group(G);
        });
    };
    // Mode-2 step of a tile with B staged through LDS.  The four column waves
    // of a row half need the same B fragments; copied once per workgroup,
    // B costs a quarter of the L2 reads of per-wave loads, and the copies of
    // several phases are in flight at once.  A phase is one k-step of 32 rows
    // in each half (the W pairs p) for JP 16-row blocks of j2: B[j2][32 rows]
    // of both halves, hi (and lo), 64 bytes per j2 row with the 16-byte
    // pieces XOR-swizzled by (j2 row >> 2) & 3.  The buffers are the X and C
    // stages of the tile's last chunk, free once every wave has consumed
    // them; NBUF - 1 phases are in flight ahead of the one being multiplied.
    constexpr int PARTS = X3 ? 2 : 1;
    constexpr int JP = JB < 4 ? JB : 4;                  // j2 blocks per phase
    constexpr bool LDS_B = PARTS * JP >= 4;              // whole copy instructions per wave
    constexpr int PB = PARTS * JP * 2048;                // bytes per phase
    constexpr int XB = LC_XSTAGE / PB, CB = CSTAGE / PB; // phase buffers in an X / a C stage
    constexpr int NBUF = XB + CB < 4 ? XB + CB : 4;
    constexpr int NJH = JB / JP, NPH = (MB / 2) * NJH;
    constexpr int CPB = LDS_B ? PARTS * 2 * JP / 8 : 1;  // copy instructions per wave and phase
    static_assert(!LDS_B || (NBUF >= 2 && XB * PB == LC_XSTAGE && CB >= 1 && 8 * CPB == PARTS * 2 * JP),
                  "mode-2 phase buffers");
    // copy instruction k of this wave fills phase rows 16 i .. 16 i + 15 with
    // i = wave + 8 k: part i / (2 JP), half (i / JP) % 2, j2 rows (i % JP) * 16 +
    // lane / 4; lane l loads logical piece (l % 4) ^ ((row >> 2) & 3)
    uint32_t bofs[CPB];
    {
        const int r = lane >> 2, piece = (lane & 3) ^ ((r >> 2) & 3);
#pragma unroll
        for (int k = 0; k < CPB; ++k) {
            const int i = wave + 8 * k;
            bofs[k] = uint32_t((jbase * 16 + (i % JP) * 16 + r) * a.ldb * 2 + piece * 16);
        }
    }
    // per-lane LDS offset of the B fragment words: row wr * JP * 16 + l16
    const uint32_t brd = uint32_t((wr * JP * 16 + l16) * 64 + ((g ^ ((l16 >> 2) & 3)) << 4));
    auto mode2_lds = [&](int64_t t, bool live, uint32_t xs_done, uint32_t cs_done) __attribute__((always_inline)) {
        constexpr int PAIRS = MB / 2;
        u32x4 wh[PAIRS][NBW], wl[PAIRS][NBW];
#pragma unroll
        for (int p = 0; p < PAIRS; ++p)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const float v[8] = {wacc[2 * p][nb][0], wacc[2 * p][nb][1], wacc[2 * p][nb][2], wacc[2 * p][nb][3],
                                    wacc[2 * p + 1][nb][0], wacc[2 * p + 1][nb][1], wacc[2 * p + 1][nb][2],
                                    wacc[2 * p + 1][nb][3]};
                if constexpr (X3) bf16_split8(v, wh[p][nb], &wl[p][nb]);
                else wh[p][nb] = bf16_round8(v);
            }
        // byte column of each half's rows in B; a half past the range copies
        // (and ignores) columns 0..127, which exist in every row of B
        const int64_t hb = row_begin + t * LC_TM;
        const uint32_t colb[2] = {uint32_t(hb * 2), hb + RW < row_end ? uint32_t((hb + RW) * 2) : 0u};
        const char *bsrc[2] = {static_cast<const char *>(a.Bhi), static_cast<const char *>(X3 ? a.Blo : a.Bhi)};
        auto buf = [&](int b) __attribute__((always_inline)) -> uint32_t {
            return b < XB ? xs_done + uint32_t(b * PB) : cs_done + uint32_t((b - XB) * PB);
        };
        auto issue = [&](auto PH) __attribute__((always_inline)) {
            constexpr int ph = decltype(PH)::value, p = ph / NJH, jh = ph % NJH;
            const uint32_t dst = buf(ph % NBUF);
#pragma unroll
            for (int k = 0; k < CPB; ++k) {
                const int i = wave + 8 * k;
                const char *src = bsrc[i / (2 * JP)] + colb[(i / JP) & 1] + int64_t(jh * JP * 16) * a.ldb * 2 + 64 * p;
                dma16s_to_lds_m0(src, bofs[k], dst + uint32_t(i * 1024));
            }
        };
        // every wave has consumed the chunk's X and C stages
        __builtin_amdgcn_s_barrier();
        static_for<NBUF - 1>([&](auto I) __attribute__((always_inline)) {
            if constexpr (decltype(I)::value < NPH) issue(I);
        });
        static_for<NPH>([&](auto PH) __attribute__((always_inline)) {
            constexpr int ph = decltype(PH)::value, p = ph / NJH, jh = ph % NJH;
            constexpr int last = ph + NBUF - 2 < NPH - 1 ? ph + NBUF - 2 : NPH - 1;
            // this wave's copies of phase ph (and of everything issued
            // before them) have landed; after the barrier, every wave's have,
            // and every wave is done with phase ph - 1's buffer
            wait_vmcnt<CPB * (last - ph)>();
            __builtin_amdgcn_s_barrier();
            if constexpr (ph + NBUF - 1 < NPH) issue(std::integral_constant<int, ph + NBUF - 1>{});
            if (live) {
                const uint32_t ba = buf(ph % NBUF) + brd;
                u32x4 fr[JP][PARTS];
                static_for<JP * PARTS>([&](auto R) __attribute__((always_inline)) {
                    constexpr int rr = decltype(R)::value, jj = rr / PARTS, part = rr % PARTS;
                    fr[jj][part] = lds_read16_at<part * JP * 2048 + jj * 1024>(ba);
                });
                static_for<JP>([&](auto JJ) __attribute__((always_inline)) {
                    constexpr int jj = decltype(JJ)::value;
                    lds_wait<(JP - 1 - jj) * PARTS>();
                    lds_dep(fr[jj][0]);
                    if constexpr (X3) lds_dep(fr[jj][PARTS - 1]);
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) {
                        auto &acc = vacc[jh * JP + jj][nb];
                        acc = mfma_bf16(fr[jj][0], wh[p][nb], acc);
                        if constexpr (X3) {
                            acc = mfma_bf16(fr[jj][0], wl[p][nb], acc);
                            acc = mfma_bf16(fr[jj][PARTS - 1], wh[p][nb], acc);
                        }
                    }
                });
            }
        });
    };
    auto tile_end = [&](int64_t t, uint32_t xs_done, uint32_t cs_done) __attribute__((always_inline)) {
        const int64_t wrow0 = row_begin + t * LC_TM + wr * RW;
        // a row half that starts past the range (the upper half of a partial
        // last tile) contributes nothing and reads no B: its columns could lie
        // past the padded row stride of B, which is a multiple of 128 only
        const bool live = wrow0 < row_end;
        if (live && wrow0 + RW > row_end) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool dead = wrow0 + mb * 16 + TR::acc_row(g, r) >= row_end;
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb)
                        if (dead) wacc[mb][nb][r] = 0.f;
                }
        }
        // rows past the range in this half contribute zeros; B's padded
        // columns up to the next multiple of 128 are zeros
        if constexpr (LDS_B) {
            mode2_lds(t, live, xs_done, cs_done);
        } else {
            if (live) slab_mode2_pipe<MATH, MB, NBW, JB>(vacc, wacc, a, jbase, wrow0, l16, g);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) wacc[mb][nb] = zero_accv<accv_t>();
    };

    // chunk q = t nk + kc: tile t, k-chunk kc.  The copies run ahead of the
    // work: X two chunks (coordinates tx, kx), C one chunk (kcn).  C's copies
    // are issued right after the barrier; X's are spread between the
    // matrix-core groups of the chunk (one after every second group), so that
    // a wave whose copy waits for room in the memory pipeline has products in
    // flight.
    const int nkc = int(nk);
    int64_t tx = 0;
    int kx = 0, kcn = 0;
    auto next_c = [&](uint32_t stage) __attribute__((always_inline)) {
        copy_c(stage, kcn);
        if (++kcn == nkc) kcn = 0;
    };
    static_assert(2 * XOPS <= NKG * MB, "one X copy per two groups");
    if (nq > 0) {
        set_x_offsets(row_begin);
        copy_x(xlds, 0, 0);
        next_c(clds);
        if (nq > 1) {
            if (nkc == 1) set_x_offsets(row_begin + LC_TM);
            copy_x(xlds + LC_XSTAGE, nkc == 1 ? 1 : 0, nkc == 1 ? 0 : 1);
        }
        tx = nkc <= 2 ? (nkc == 1 ? 2 : 1) : 0;
        kx = nkc <= 2 ? 0 : 2;
    }
    int64_t t = 0;
    int kc = 0, xst = 0, cst = 0;
    for (int64_t q = 0; q < nq; ++q) {
        // chunk q landed everywhere: this wave's copies of X(q) and C(q) are
        // done when at most its copies of X(q + 1) are outstanding
        if (q + 1 < nq) wait_vmcnt<XOPS>();
        else wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        if (q + 1 < nq) next_c(clds + uint32_t((cst ^ 1) * CSTAGE));
        const bool x_next = q + 2 < nq, last_of_tile = kc == nkc - 1;
        const uint32_t xstage = xlds + uint32_t((xst == 0 ? 2 : xst - 1) * LC_XSTAGE);
        const char *xb = xslab;
        if (x_next) {
            if (kx == 0) set_x_offsets(row_begin + tx * LC_TM);
            xb = xslab + (row_begin + tx * LC_TM) * xrow_bytes + kx * 128;
        }
        const uint32_t xs = xlds + uint32_t(xst * LC_XSTAGE), cs = clds + uint32_t(cst * CSTAGE);
        compute(xs, cs, [&](auto G) __attribute__((always_inline)) {
            constexpr int g = decltype(G)::value;
            if constexpr (g % 2 == 1 && g / 2 < XOPS)
                if (x_next) dma16s_to_lds_m0(xb, xlo[g / 2], xstage + uint32_t((wave * XOPS + g / 2) * 1024));
        });
        if (last_of_tile) {
            tile_end(t, xs, cs);
            kc = 0;
            ++t;
        } else {
            ++kc;
        }
        if (x_next && ++kx == nkc) { kx = 0; ++tx; }
        xst = xst == 2 ? 0 : xst + 1;
        cst ^= 1;
    }

    // the upper row half adds its V partial to the lower one's through LDS
    // (every chunk has been consumed: the X stages are free)
    constexpr int NV = JB * NBW * 4;
    constexpr int PER_STAGE = LC_XSTAGE / 4 / 256;  // floats of one (wc, lane) slot per stage
    static_assert(NV <= 2 * PER_STAGE, "reduction buffer");
    __syncthreads();
    auto slot = [&](int v) __attribute__((always_inline)) -> float * {   // v-th value of this (wc, lane)
        float *base = reinterpret_cast<float *>(xbuf + (v < PER_STAGE ? 0 : LC_XSTAGE));
        return base + ((v % PER_STAGE) * 4 + wc) * 64 + lane;
    };
    if (wr == 1) {
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) *slot((jb * NBW + nb) * 4 + r) = vacc[jb][nb][r];
    }
    __syncthreads();
    if (wr != 0) return;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) vacc[jb][nb][r] += *slot((jb * NBW + nb) * 4 + r);

    float *Vp = static_cast<float *>(a.V) + (i1 * a.P + s) * a.J2pad * a.J3pad;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j2 = int64_t(jbase + jb) * 16 + TR::acc_row(g, r);
                Vp[j2 * a.J3pad + colb + wc * NBW * 16 + nb * 16 + l16] = vacc[jb][nb][r];
            }
}

// ---------------------------------------------------------------------------
// Mode-1 contraction with partial sums:
//   Y[j1, n] = sum_i1 A[j1, i1] * sum_p V[i1][p][n],   n = j2 * J3pad + j3.
// A workgroup owns 64 columns n and up to 128 rows j1 (grid.z tiles larger
// J1); grid.y splits the i1 range.  V is streamed once:
// each lane reads one column over VE consecutive rows (a wave reads 256
// contiguous bytes per row), converts to the operand format and stores the
// VE values as one 16-byte LDS word, k-contiguous, which is exactly the
// k-slot fragment the B operand wants.  With one split the result goes to Y;
// otherwise to per-split partials summed by k_mode1_reduce.
// ---------------------------------------------------------------------------
struct Mode1Args {
    const void *Ahi, *Alo;   // [J1pad][lda]
    int64_t lda;
    const void *V;           // [I1][P][NN]
    int64_t I1;
    int P;
    int64_t NN, J3pad;
    void *Y;                 // final output, used when KS == 1
    void *Ypart;             // [KS][J1pad][NN] partials, used when KS > 1
    int64_t J1, J2, J3, J1pad;
    int KS;
    int64_t rows_per_split;
};

template <int MATH>
struct Mode1Cfg {
    typedef MathTraits<MATH> TR;
    typedef typename TR::lds_t LT;
    static constexpr int VE = TR::VE, KG = TR::KG;
    static constexpr int KT = 2 * KG;                                  // rows per chunk
    static constexpr int ROWB = KT * int(sizeof(LT)) + 16;             // LDS stride per column
    static constexpr int BUFB = 64 * ROWB;
    static constexpr int ITEMS = KT * 64 / (256 * VE);                 // 16-byte words per thread per chunk
    static constexpr bool SPLIT = (MATH == M_BF16X3);
};

// MW 16-row blocks and NW 16-column blocks per wave.  NW == 4: the waves
// split the rows (wave w: blocks w*MW ..), each covering all 64 columns, so
// every element of A is fetched once per workgroup; NW == 1: the waves split
// the columns (small J1).
template <int MATH, int MW, int NW>
__global__ void __launch_bounds__(256) k_mode1(const Mode1Args a) {
    typedef Mode1Cfg<MATH> CF;
    typedef MathTraits<MATH> TR;
    typedef typename TR::accv_t accv_t;
    typedef typename TR::acc_t acc_t;
    typedef typename TR::fac_t FT;
    constexpr int VE = CF::VE, KG = CF::KG, KT = CF::KT, ITEMS = CF::ITEMS;
    __shared__ __align__(16) unsigned char lds[2 * CF::BUFB * (CF::SPLIT ? 2 : 1)];
    unsigned char *lhi = lds, *llo = lds + 2 * CF::BUFB;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t n0 = int64_t(blockIdx.x) * 64;
    const int ks = int(blockIdx.y);
    const int64_t kb = int64_t(ks) * a.rows_per_split;
    const int64_t ke = a.I1 < kb + a.rows_per_split ? a.I1 : kb + a.rows_per_split;
    const int64_t nch = ke > kb ? ceil_div(ke - kb, KT) : 0;
    const acc_t *V = static_cast<const acc_t *>(a.V);
    const FT *Ah = static_cast<const FT *>(a.Ahi);
    const FT *Al = static_cast<const FT *>(a.Alo);

    // loader: thread (column c = tid % 64, word w = tid / 64 + 4*item) covers rows VE*w .. VE*w+VE-1
    const int lc = tid & 63, lw = tid >> 6;
    // V chunks in flight in registers: two ahead of the one being computed
    // (slots ch % 2), one ahead for bf16x3 with two row blocks per wave
    acc_t pre2[2][ITEMS][VE];
    // all ITEMS*VE loads of one partial are independent and issued together;
    // rows past the range read row kb (valid) and are zeroed
    auto fetch = [&](int64_t ch, acc_t (&pre)[ITEMS][VE]) __attribute__((always_inline)) {
        const int64_t r0 = kb + ch * KT;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it)
#pragma unroll
            for (int e = 0; e < VE; ++e) pre[it][e] = acc_t(0);
        for (int p = 0; p < a.P; ++p) {
            const acc_t *vp = V + int64_t(p) * a.NN + n0 + lc;
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    const int64_t k = r0 + (lw + 4 * it) * VE + e;
                    const acc_t v = vp[(k < ke ? k : kb) * a.P * a.NN];
                    pre[it][e] += k < ke ? v : acc_t(0);
                }
        }
    };
    auto store = [&](int buf, const acc_t (&pre)[ITEMS][VE]) __attribute__((always_inline)) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int off = buf * CF::BUFB + lc * CF::ROWB + (lw + 4 * it) * 16;
            if constexpr (MATH == M_F32) {
                *reinterpret_cast<f32x4 *>(lhi + off) = f32x4{pre[it][0], pre[it][1], pre[it][2], pre[it][3]};
            } else if constexpr (MATH == M_F64) {
                *reinterpret_cast<f64x2 *>(lhi + off) = f64x2{pre[it][0], pre[it][1]};
            } else {
                const float v[8] = {pre[it][0], pre[it][1], pre[it][2], pre[it][3],
                                    pre[it][4], pre[it][5], pre[it][6], pre[it][7]};
                u32x4 h, l;
                if constexpr (CF::SPLIT) {
                    bf16_split8(v, h, &l);
                    *reinterpret_cast<u32x4 *>(llo + off) = l;
                } else {
                    h = bf16_round8(v);
                }
                *reinterpret_cast<u32x4 *>(lhi + off) = h;
            }
        }
    };

    constexpr int MBW = NW == 4 ? 4 * MW : MW;          // 16-row blocks per workgroup
    const int mbase = NW == 4 ? wave * MW : 0;
    const int nbase = NW == 4 ? 0 : wave;
    const int64_t m0 = int64_t(blockIdx.z) * MBW * 16;
    accv_t acc[MW][NW];
#pragma unroll
    for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j) acc[i][j] = zero_accv<accv_t>();

    // A's fragments of a chunk are loaded one chunk ahead and before the next
    // chunk's V prefetch: vector-memory loads complete in order, so a wait for
    // A issued after the prefetch would also wait for the prefetch's HBM trip
    V16 fah[MW][2], fal[MW][2];
    auto load_a = [&](int64_t ch) __attribute__((always_inline)) {
#pragma unroll
        for (int kg = 0; kg < 2; ++kg) {
            const int64_t k0 = kb + ch * KT + kg * KG + g * VE;
#pragma unroll
            for (int i = 0; i < MW; ++i) {
                const int64_t off = (m0 + (mbase + i) * 16 + l16) * a.lda + k0;
                fah[i][kg] = ld16(Ah + off);
                if constexpr (CF::SPLIT) fal[i][kg] = ld16(Al + off);
            }
        }
    };
    auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int kg = 0; kg < 2; ++kg) {
            V16 bh[NW], bl[NW];
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const int loff = buf * CF::BUFB + ((nbase + j) * 16 + l16) * CF::ROWB + kg * 64 + g * 16;
                bh[j].u = *reinterpret_cast<const u32x4 *>(lhi + loff);
                if constexpr (CF::SPLIT) bl[j].u = *reinterpret_cast<const u32x4 *>(llo + loff);
            }
#pragma unroll
            for (int i = 0; i < MW; ++i) {
                const V16 ah = fah[i][kg];
                V16 al;
                if constexpr (CF::SPLIT) al = fal[i][kg];
#pragma unroll
                for (int j = 0; j < NW; ++j) {
                    mma_kgroup<MATH == M_BF16X3 ? M_BF16 : MATH>(acc[i][j], ah, bh[j]);
                    if constexpr (CF::SPLIT) {
                        mma_kgroup<M_BF16>(acc[i][j], ah, bl[j]);
                        mma_kgroup<M_BF16>(acc[i][j], al, bh[j]);
                    }
                }
            }
        }
    };
    // one chunk: prefetch chunk ch + 2 into the slot chunk ch left, compute
    // chunk ch, then store chunk ch + 1 (slot 1 - S) and load its A fragments
    auto step = [&](int64_t ch, auto SLOT) __attribute__((always_inline)) {
        constexpr int S = decltype(SLOT)::value;
        if (ch + 2 < nch) fetch(ch + 2, pre2[S]);
        compute(S);
        if (ch + 1 < nch) {
            store(1 - S, pre2[1 - S]);
            load_a(ch + 1);
        }
        __syncthreads();
    };
    if constexpr (CF::SPLIT && MW == 2) {
        // bf16x3 with two row blocks per wave: one chunk ahead (two would take
        // the registers of a third resident wave per SIMD, measured slower)
        if (nch > 0) {
            fetch(0, pre2[0]);
            store(0, pre2[0]);
            load_a(0);
        }
        __syncthreads();
        for (int64_t ch = 0; ch < nch; ++ch) {
            if (ch + 1 < nch) fetch(ch + 1, pre2[0]);
            compute(int(ch & 1));
            if (ch + 1 < nch) {
                store(int((ch + 1) & 1), pre2[0]);
                load_a(ch + 1);
            }
            __syncthreads();
        }
    } else {
        if (nch > 0) {
            fetch(0, pre2[0]);
            if (nch > 1) fetch(1, pre2[1]);
            store(0, pre2[0]);
            load_a(0);
        }
        __syncthreads();
        for (int64_t ch = 0; ch < nch; ch += 2) {
            step(ch, std::integral_constant<int, 0>{});
            if (ch + 1 < nch) step(ch + 1, std::integral_constant<int, 1>{});
        }
    }

    acc_t *Y = static_cast<acc_t *>(a.Y);
    acc_t *Yp = static_cast<acc_t *>(a.Ypart) + int64_t(ks) * a.J1pad * a.NN;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        const int64_t n = n0 + (nbase + j) * 16 + l16;
        const int64_t j2 = n / a.J3pad, j3 = n % a.J3pad;
#pragma unroll
        for (int i = 0; i < MW; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j1 = m0 + (mbase + i) * 16 + TR::acc_row(g, r);
                if (a.KS == 1) {
                    if (j1 < a.J1 && j2 < a.J2 && j3 < a.J3) Y[(j1 * a.J2 + j2) * a.J3 + j3] = acc[i][j][r];
                } else {
                    Yp[j1 * a.NN + n] = acc[i][j][r];
                }
            }
    }
}

// Y[j1][j2][j3] = sum_ks Ypart[ks][j1][j2 * J3pad + j3] in increasing ks order.
// Workgroup r owns the row (j1, j2) = (r / J2, r % J2) (one scalar division
// per workgroup instead of three per element), its lanes the j3.
template <typename T>
__global__ void __launch_bounds__(64) k_mode1_reduce(const Mode1Args a) {
    const int64_t row = blockIdx.x;
    const int64_t j1 = row / a.J2, j2 = row - j1 * a.J2;
    const T *Yp = static_cast<const T *>(a.Ypart) + j1 * a.NN + j2 * a.J3pad;
    T *Y = static_cast<T *>(a.Y) + row * a.J3;
    const int64_t ps = a.J1pad * a.NN;
    for (int64_t j3 = threadIdx.x; j3 < a.J3; j3 += 64) {
        const T *p = Yp + j3;
        T s = T(0);
        int k = 0;
        for (; k + 4 <= a.KS; k += 4) {   // four loads in flight, summed in order
            const T v0 = p[k * ps], v1 = p[(k + 1) * ps], v2 = p[(k + 2) * ps], v3 = p[(k + 3) * ps];
            s += v0; s += v1; s += v2; s += v3;
        }
        for (; k < a.KS; ++k) s += p[k * ps];
        Y[j3] = s;
    }
}

// The same sum, 16 bytes per lane: thread t owns four consecutive j3 of row
// t / (J3 / 4) (needs J3 % 4 == 0; J3pad and NN are multiples of 16, so every
// access is 16-byte aligned).  Same order of the terms as k_mode1_reduce.
__global__ void __launch_bounds__(256) k_mode1_reduce4(const Mode1Args a) {
    const int q4 = int(a.J3 / 4);
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= a.J1 * a.J2 * q4) return;
    const int64_t row = t / q4, q = t - row * q4;
    const int64_t j1 = row / a.J2, j2 = row - j1 * a.J2;
    const float *p = static_cast<const float *>(a.Ypart) + j1 * a.NN + j2 * a.J3pad + 4 * q;
    const int64_t ps = a.J1pad * a.NN;
    f32x4 s = *reinterpret_cast<const f32x4 *>(p);
    int k = 1;
    for (; k + 4 <= a.KS; k += 4) {   // four loads in flight, summed in order
        const f32x4 v0 = *reinterpret_cast<const f32x4 *>(p + k * ps);
        const f32x4 v1 = *reinterpret_cast<const f32x4 *>(p + (k + 1) * ps);
        const f32x4 v2 = *reinterpret_cast<const f32x4 *>(p + (k + 2) * ps);
        const f32x4 v3 = *reinterpret_cast<const f32x4 *>(p + (k + 3) * ps);
        s += v0; s += v1; s += v2; s += v3;
    }
    for (; k < a.KS; ++k) s += *reinterpret_cast<const f32x4 *>(p + k * ps);
    *reinterpret_cast<f32x4 *>(static_cast<float *>(a.Y) + row * a.J3 + 4 * q) = s;
}

// ---------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------
struct ChainPlan {
    int math, xdt;
    int WC, NBW, WR, JBMAX, JB, MBK, m1_MW, m1_NW;
    int64_t cols;                 // j3 columns per workgroup
    int64_t J3pad, J2pad, J1pad;
    int64_t n_j3_tiles, n_j2_tiles, n_m1_tiles;
    int KS;                       // i1 splits of the mode-1 kernel
    int64_t m1_rows_per_split;
    int S, P;
    int64_t rows_per_split;
    int64_t ldc, ldb, lda;
    size_t fsz;                   // bytes per factor operand element
    size_t acc_sz;
    size_t off_Chi, off_Clo, off_Bhi, off_Blo, off_Ahi, off_Alo, off_V, off_Yp, total;
    bool split;                   // factors need hi/lo
};

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

static bool combo_ok(int x, int f, int y, int m) {
    if (m == TTM_MATH_F64) return x == TTM_F64 && f == TTM_F64 && y == TTM_F64;
    if (f != TTM_F32 || y != TTM_F32) return false;
    if (m == TTM_MATH_F32 || m == TTM_MATH_BF16 || m == TTM_MATH_BF16X3) return x == TTM_F32 || x == TTM_BF16;
    return false;
}

static bool make_plan(const ttm_shape &s, int xdt, int math, ChainPlan &p) {
    p = ChainPlan();
    p.math = math;
    p.xdt = xdt;
    const int64_t I1 = s.I[0], I2 = s.I[1], I3 = s.I[2];
    const int64_t J1 = s.J[0], J2 = s.J[1], J3 = s.J[2];
    const bool bf = (math == TTM_MATH_BF16 || math == TTM_MATH_BF16X3);
    const int KG = math == TTM_MATH_F64 ? 8 : (math == TTM_MATH_F32 ? 16 : 32);
    const int KC = 2 * KG;
    p.split = (math == TTM_MATH_BF16X3);
    p.fsz = math == TTM_MATH_F64 ? 8 : (bf ? 2 : 4);
    p.acc_sz = math == TTM_MATH_F64 ? 8 : 4;

    // columns (j3) per workgroup and how the 4 waves share them
    const int64_t J3r = round_up(J3, 16);
    if (J3r <= 16) { p.WC = 1; p.NBW = 1; }
    else if (J3r <= 32) { p.WC = 2; p.NBW = 1; }
    else if (J3r <= 64 || math == TTM_MATH_F64) { p.WC = 4; p.NBW = 1; }
    else { p.WC = 4; p.NBW = 2; }
    p.WR = 4 / p.WC;
    p.cols = int64_t(p.WC) * p.NBW * 16;
    p.n_j3_tiles = ceil_div(J3r, p.cols);
    p.J3pad = p.n_j3_tiles * p.cols;
    p.JBMAX = math == TTM_MATH_F64 ? 4 : 8;
    {
        const int64_t jbn = ceil_div(J2, 16);
        p.JB = jbn >= p.JBMAX ? p.JBMAX : (jbn > 2 ? 4 : (jbn > 1 ? 2 : 1));
    }
    p.n_j2_tiles = ceil_div(ceil_div(J2, 16), p.JB);
    p.J2pad = p.n_j2_tiles * p.JB * 16;

    // split the i2 rows of a slab so the grid has enough workgroups
    const int64_t base = I1 * p.n_j3_tiles * p.n_j2_tiles;
    const int64_t max_s = ceil_div(I2, SLAB_TM);
    int64_t S = ceil_div(1024, base);
    if (S < 1) S = 1;
    if (S > max_s) S = max_s;
    if (S > 64) S = 64;
    p.rows_per_split = round_up(ceil_div(I2, S), SLAB_TM);
    p.S = int(ceil_div(I2, p.rows_per_split));
    p.P = p.S * p.WR;

    // mode-1 kernel tiling: MW row blocks and NW column blocks per wave
    const int64_t J1b = ceil_div(J1, 16);
    if (J1b <= 2) { p.m1_NW = 1; p.m1_MW = int(J1b); }
    else { p.m1_NW = 4; p.m1_MW = J1b >= 5 ? 2 : 1; }
    p.MBK = p.m1_NW == 4 ? 4 * p.m1_MW : p.m1_MW;
    p.n_m1_tiles = ceil_div(J1b, p.MBK);
    p.J1pad = p.n_m1_tiles * p.MBK * 16;

    p.ldc = round_up(I3, KC);
    p.ldb = round_up(I2, SLAB_TM);
    p.lda = round_up(I1, KC);

    // mode-1 kernel: split the i1 range while the column tiles alone leave the
    // GPU short of workgroups (about 512 in all: measured at 1024^3 -> 128^3,
    // fewer, longer splits beat about 1024 once V is prefetched ahead),
    // keeping the partials at most half of V's size
    {
        const int64_t NN = p.J2pad * p.J3pad;
        const int64_t wg = (NN / 64) * p.n_m1_tiles;
        int64_t ks = ceil_div(512, wg);
        const int64_t ks_bytes = (I1 * p.P) / (2 * p.J1pad);
        if (ks > ks_bytes) ks = ks_bytes;
        if (ks > ceil_div(I1, KC)) ks = ceil_div(I1, KC);
        if (ks > 64) ks = 64;
        if (ks < 1) ks = 1;
        p.m1_rows_per_split = round_up(ceil_div(I1, ks), KC);
        p.KS = int(ceil_div(I1, p.m1_rows_per_split));
    }

    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = al256(off + bytes); return o; };
    p.off_Chi = take(size_t(p.J3pad) * p.ldc * p.fsz);
    p.off_Clo = p.split ? take(size_t(p.J3pad) * p.ldc * p.fsz) : 0;
    p.off_Bhi = take(size_t(p.J2pad) * p.ldb * p.fsz);
    p.off_Blo = p.split ? take(size_t(p.J2pad) * p.ldb * p.fsz) : 0;
    p.off_Ahi = take(size_t(p.J1pad) * p.lda * p.fsz);
    p.off_Alo = p.split ? take(size_t(p.J1pad) * p.lda * p.fsz) : 0;
    p.off_V = take(size_t(I1) * p.P * p.J2pad * p.J3pad * p.acc_sz);
    p.off_Yp = p.KS > 1 ? take(size_t(p.KS) * p.J1pad * p.J2pad * p.J3pad * p.acc_sz) : 0;
    p.total = off;
    // launch-grid limits
    if (I1 * p.S > 0x7fffffffLL || p.n_j3_tiles > 65535 || p.n_j2_tiles > 65535 || p.n_m1_tiles > 65535 ||
        p.J2pad * p.J3pad / 64 > 0x7fffffffLL || p.KS > 65535 || J1 * J2 > 0x7fffffffLL)
        return false;
    return true;
}

template <int MATH, typename XT, int WC, int NBW, int JB>
static int launch_slab(const ChainPlan &p, const SlabArgs &a, hipStream_t st) {
    typedef SlabCfg<MATH, XT> CF;
    dim3 grid(unsigned(a.I1 * a.S), unsigned(p.n_j3_tiles), unsigned(p.n_j2_tiles));
    const size_t lds = CF::lds_bytes();
    static std::atomic<uint64_t> attr_set{0};
    if (int rc = ensure_lds_limit(reinterpret_cast<const void *>(&k_slab<MATH, XT, WC, NBW, JB>), lds, attr_set))
        return rc;
    return launch("ttm_slab", st, [&] {
        hipLaunchKernelGGL((k_slab<MATH, XT, WC, NBW, JB>), grid, dim3(SLAB_THREADS), lds, st, a);
    });
}

// Which direct-to-LDS variant applies (0: none): 16-byte aligned rows and
// whole chunks along i3.  The two-stage kernel (256-byte chunks, returned as
// 256) needs X already in the operand format; the kernel with C in LDS
// (returned as 128) takes bf16 X with the bf16 forms and four column waves.
// Automatic selection takes the kernel with C in LDS where it applies and the
// row range of a workgroup holds at least one whole 256-row tile (measured at
// 1024^3 -> 128^3 it runs 15% ahead of the two-stage kernel with bf16x3 and
// 7% with bf16; with 128-row ranges, as at 256^3 -> 64^3, half of each tile
// is padding), then the two-stage kernel where X is in the operand format,
// and the register-staged kernel otherwise.
template <int MATH, typename XT, int WC>
static int dma_rowbytes(const SlabArgs &a) {
    typedef typename MathTraits<MATH>::lds_t LT;
    const int mode = slab_kernel_mode();
    if (mode == 1 || !a.x_vec || !aligned(a.X, 16)) return 0;
    const int64_t es = int64_t(sizeof(XT));
    if (mode == 0 || mode == 3) {                            // C through LDS where it applies
        if constexpr (WC == 4 && (MATH == M_BF16 || MATH == M_BF16X3) && std::is_same<XT, uint16_t>::value)
            if (a.I3 % 64 == 0 && a.ldc % 64 == 0 && a.I3 <= (int64_t(1) << 22) && a.ldc <= (int64_t(1) << 22) &&
                a.J2pad * a.ldb < (int64_t(1) << 30) &&
                aligned(a.Chi, 16) && (!a.Clo || aligned(a.Clo, 16)) &&
                (mode == 3 || a.rows_per_split >= LC_TM))
                return 128;
        if (mode == 3) return 0;
    }
    if constexpr (!std::is_same<XT, LT>::value) return 0;
    return a.I3 % (256 / es) == 0 ? 256 : 0;
}

template <int MATH, typename XT, int WC, int NBW, int JB>
static int launch_slab_dma_rb(const ChainPlan &p, const SlabArgs &a, int rb, hipStream_t st) {
    typedef typename MathTraits<MATH>::lds_t LT;
    dim3 grid(unsigned(a.I1 * a.S), unsigned(p.n_j3_tiles), unsigned(p.n_j2_tiles));
    if constexpr (std::is_same<XT, LT>::value) {
        if (rb == 256)
            return launch("ttm_slab", st, [&] {
                hipLaunchKernelGGL((k_slab_dma<MATH, WC, NBW, JB>), grid, dim3(SLAB_THREADS), 0, st, a);
            });
    }
    if constexpr (WC == 4 && (MATH == M_BF16 || MATH == M_BF16X3) && std::is_same<XT, uint16_t>::value) {
        if (rb == 128)
            return launch("ttm_slab", st, [&] {
                hipLaunchKernelGGL((k_slab_lc<MATH, NBW, JB>), grid, dim3(LC_THREADS), 0, st, a);
            });
    }
    return TTM_ERR_UNSUPPORTED;
}

template <int MATH, typename XT, int WC, int NBW>
static int dispatch_slab_jb(const ChainPlan &p, const SlabArgs &a, hipStream_t st) {
    if (const int rb = dma_rowbytes<MATH, XT, WC>(a)) {
        switch (p.JB) {
            case 1: return launch_slab_dma_rb<MATH, XT, WC, NBW, 1>(p, a, rb, st);
            case 2: return launch_slab_dma_rb<MATH, XT, WC, NBW, 2>(p, a, rb, st);
            case 4: return launch_slab_dma_rb<MATH, XT, WC, NBW, 4>(p, a, rb, st);
            default:
                if constexpr (MATH != M_F64) return launch_slab_dma_rb<MATH, XT, WC, NBW, 8>(p, a, rb, st);
                return TTM_ERR_UNSUPPORTED;
        }
    }
    switch (p.JB) {
        case 1: return launch_slab<MATH, XT, WC, NBW, 1>(p, a, st);
        case 2: return launch_slab<MATH, XT, WC, NBW, 2>(p, a, st);
        case 4: return launch_slab<MATH, XT, WC, NBW, 4>(p, a, st);
        default:
            if constexpr (MATH != M_F64) return launch_slab<MATH, XT, WC, NBW, 8>(p, a, st);
            return TTM_ERR_UNSUPPORTED;
    }
}

template <int MATH, typename XT>
static int dispatch_slab(const ChainPlan &p, const SlabArgs &a, hipStream_t st) {
    if (p.WC == 1) return dispatch_slab_jb<MATH, XT, 1, 1>(p, a, st);
    if (p.WC == 2) return dispatch_slab_jb<MATH, XT, 2, 1>(p, a, st);
    if (p.NBW == 1) return dispatch_slab_jb<MATH, XT, 4, 1>(p, a, st);
    if constexpr (MATH != M_F64) return dispatch_slab_jb<MATH, XT, 4, 2>(p, a, st);
    return TTM_ERR_UNSUPPORTED;
}

template <int MATH>
static int dispatch_mode1(const ChainPlan &p, const Mode1Args &a, hipStream_t st) {
    typedef typename MathTraits<MATH>::acc_t acc_t;
    dim3 grid(unsigned(p.J2pad * p.J3pad / 64), unsigned(p.KS), unsigned(p.n_m1_tiles));
    auto go = [&](auto kern) {
        return launch("ttm_mode1", st, [&] { hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a); });
    };
    int rc;
    if (p.m1_NW == 1) rc = p.m1_MW == 1 ? go(k_mode1<MATH, 1, 1>) : go(k_mode1<MATH, 2, 1>);
    else rc = p.m1_MW == 1 ? go(k_mode1<MATH, 1, 4>) : go(k_mode1<MATH, 2, 4>);
    if (rc || p.KS == 1) return rc;
    if (MATH != M_F64 && a.J3 % 4 == 0 && aligned(a.Y, 16)) {
        const int64_t n4 = a.J1 * a.J2 * (a.J3 / 4);
        return launch("ttm_mode1_reduce", st, [&] {
            hipLaunchKernelGGL(k_mode1_reduce4, dim3(unsigned(ceil_div(n4, 256))), dim3(256), 0, st, a);
        });
    }
    return launch("ttm_mode1_reduce", st, [&] {
        hipLaunchKernelGGL((k_mode1_reduce<acc_t>), dim3(unsigned(a.J1 * a.J2)), dim3(64), 0, st, a);
    });
}

template <int MATH>
static int run_chain(const ChainPlan &p, const ttm_shape &s, const void *X, const void *A, const void *B,
                     const void *C, void *Y, unsigned char *ws, hipStream_t st) {
    // 1. factor operands
    PrepArgs pa;
    const void *src[3] = {A, B, C};
    const size_t offh[3] = {p.off_Ahi, p.off_Bhi, p.off_Chi}, offl[3] = {p.off_Alo, p.off_Blo, p.off_Clo};
    const int64_t Jpad[3] = {p.J1pad, p.J2pad, p.J3pad}, ld[3] = {p.lda, p.ldb, p.ldc};
    int64_t maxn = 0;
    for (int f = 0; f < 3; ++f) {
        pa.src[f] = src[f];
        pa.hi[f] = ws + offh[f];
        pa.lo[f] = p.split ? ws + offl[f] : nullptr;
        pa.J[f] = s.J[f];
        pa.I[f] = s.I[f];
        pa.Jpad[f] = Jpad[f];
        pa.ld[f] = ld[f];
        pa.perm32[f] = (f == 1 && (MATH == M_BF16 || MATH == M_BF16X3)) ? 1 : 0;
        maxn = std::max<int64_t>(maxn, Jpad[f] * ld[f]);
    }
    // float and double operands whose padded arrays would equal the factors
    // (rows a multiple of the tile, row length a multiple of the k chunk) are
    // read where they are: the preparation would be a plain copy
    bool direct = false;
    if constexpr (MATH == M_F32 || MATH == M_F64) {
        direct = true;
        for (int f = 0; f < 3; ++f)
            direct = direct && Jpad[f] == s.J[f] && ld[f] == s.I[f] && aligned(src[f], 16);
    }
    const void *fac[3];
    for (int f = 0; f < 3; ++f) fac[f] = direct ? src[f] : static_cast<const void *>(ws + offh[f]);
    dim3 pgrid(unsigned(std::min<int64_t>(ceil_div(maxn, 256), 4096)), 3);
    int rc = TTM_OK;
    if (!direct) {
        if constexpr (MATH == M_F64)
            rc = launch("ttm_prep", st,
                        [&] { hipLaunchKernelGGL((k_prep_factors<double, MATH>), pgrid, dim3(256), 0, st, pa); });
        else
            rc = launch("ttm_prep", st,
                        [&] { hipLaunchKernelGGL((k_prep_factors<float, MATH>), pgrid, dim3(256), 0, st, pa); });
    }
    if (rc) return rc;

    // 2. slab kernel (modes 3 and 2)
    SlabArgs sa;
    sa.X = X;
    sa.I1 = s.I[0]; sa.I2 = s.I[1]; sa.I3 = s.I[2];
    sa.Chi = fac[2]; sa.Clo = p.split ? ws + p.off_Clo : nullptr; sa.ldc = p.ldc;
    sa.Bhi = fac[1]; sa.Blo = p.split ? ws + p.off_Blo : nullptr; sa.ldb = p.ldb;
    sa.V = ws + p.off_V;
    sa.J2pad = p.J2pad; sa.J3pad = p.J3pad;
    sa.P = p.P; sa.S = p.S;
    sa.rows_per_split = p.rows_per_split;
    const size_t xsz = dtype_size(p.xdt);
    sa.x_vec = ((s.I[2] * int64_t(xsz)) % 16 == 0) && aligned(X, 16);
    if constexpr (MATH == M_F64) {
        rc = dispatch_slab<M_F64, double>(p, sa, st);
    } else if (p.xdt == TTM_BF16) {
        // bf16 X: 8-byte groups for float operands need 8-byte rows
        if constexpr (MATH == M_F32) sa.x_vec = ((s.I[2] * 2) % 8 == 0) && aligned(X, 16);
        rc = dispatch_slab<MATH, uint16_t>(p, sa, st);
    } else {
        if constexpr (MATH == M_BF16 || MATH == M_BF16X3) sa.x_vec = ((s.I[2] * 4) % 32 == 0) && aligned(X, 16);
        rc = dispatch_slab<MATH, float>(p, sa, st);
    }
    if (rc) return rc;

    // 3. mode 1
    Mode1Args ma;
    ma.Ahi = fac[0]; ma.Alo = p.split ? ws + p.off_Alo : nullptr; ma.lda = p.lda;
    ma.V = ws + p.off_V; ma.I1 = s.I[0]; ma.P = p.P;
    ma.NN = p.J2pad * p.J3pad; ma.J3pad = p.J3pad;
    ma.Y = Y; ma.Ypart = p.KS > 1 ? ws + p.off_Yp : nullptr;
    ma.J1 = s.J[0]; ma.J2 = s.J[1]; ma.J3 = s.J[2]; ma.J1pad = p.J1pad;
    ma.KS = p.KS; ma.rows_per_split = p.m1_rows_per_split;
    return dispatch_mode1<MATH>(p, ma, st);
}

static int validate_shape(const ttm_shape *s) {
    if (!s) return TTM_ERR_INVALID_ARG;
    for (int n = 0; n < 3; ++n)
        if (s->I[n] < 1 || s->J[n] < 1 || s->I[n] > (int64_t(1) << 31) || s->J[n] > (int64_t(1) << 31))
            return TTM_ERR_INVALID_ARG;
    if (checked_prod(checked_prod(s->I[0], s->I[1]), s->I[2]) < 0) return TTM_ERR_INVALID_ARG;
    if (checked_prod(checked_prod(s->J[0], s->J[1]), s->J[2]) < 0) return TTM_ERR_INVALID_ARG;
    return TTM_OK;
}

// Argument checks shared by the entry points of the chain (everything but
// the workspace) and the plan for the shape.
static int chain_check(const ttm_shape *s, const void *X, int x_dtype, const void *A, const void *B,
                       const void *C, int f_dtype, const void *Y, int y_dtype, int math, ChainPlan &p) {
    int rc = validate_shape(s);
    if (rc) return rc;
    if (!combo_ok(x_dtype, f_dtype, y_dtype, math)) return TTM_ERR_UNSUPPORTED;
    if (!X || !A || !B || !C || !Y) return TTM_ERR_INVALID_ARG;
    const size_t fs = dtype_size(f_dtype), ys = dtype_size(y_dtype), xs = dtype_size(x_dtype);
    if (!aligned(X, 16) || !aligned(Y, 16) || !aligned(A, fs) || !aligned(B, fs) || !aligned(C, fs))
        return TTM_ERR_INVALID_ARG;
    if (!make_plan(*s, x_dtype, math, p)) return TTM_ERR_UNSUPPORTED;
    const size_t ny = size_t(s->J[0] * s->J[1] * s->J[2]) * ys;
    const size_t nx = size_t(s->I[0] * s->I[1] * s->I[2]) * xs;
    if (overlaps(Y, ny, X, nx) || overlaps(Y, ny, A, size_t(s->J[0] * s->I[0]) * fs) ||
        overlaps(Y, ny, B, size_t(s->J[1] * s->I[1]) * fs) || overlaps(Y, ny, C, size_t(s->J[2] * s->I[2]) * fs))
        return TTM_ERR_ALIAS;
    return TTM_OK;
}

// Workspace checks and the launches.
static int chain_run(const ChainPlan &p, const ttm_shape *s, const void *X, const void *A, const void *B,
                     const void *C, void *Y, int math, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!ws || ws_bytes < p.total) return TTM_ERR_WORKSPACE;
    if (!aligned(ws, 16)) return TTM_ERR_INVALID_ARG;
    const size_t fs = p.math == TTM_MATH_F64 ? 8 : 4, ys = fs, xs = dtype_size(p.xdt);
    const size_t ny = size_t(s->J[0] * s->J[1] * s->J[2]) * ys;
    const size_t nx = size_t(s->I[0] * s->I[1] * s->I[2]) * xs;
    if (overlaps(Y, ny, ws, p.total) || overlaps(ws, p.total, X, nx) ||
        overlaps(ws, p.total, A, size_t(s->J[0] * s->I[0]) * fs) ||
        overlaps(ws, p.total, B, size_t(s->J[1] * s->I[1]) * fs) ||
        overlaps(ws, p.total, C, size_t(s->J[2] * s->I[2]) * fs))
        return TTM_ERR_ALIAS;
    unsigned char *w = static_cast<unsigned char *>(ws);
    switch (math) {
        case TTM_MATH_F64: return run_chain<M_F64>(p, *s, X, A, B, C, Y, w, st);
        case TTM_MATH_F32: return run_chain<M_F32>(p, *s, X, A, B, C, Y, w, st);
        case TTM_MATH_BF16: return run_chain<M_BF16>(p, *s, X, A, B, C, Y, w, st);
        case TTM_MATH_BF16X3: return run_chain<M_BF16X3>(p, *s, X, A, B, C, Y, w, st);
        default: return TTM_ERR_UNSUPPORTED;
    }
}

// ---------------------------------------------------------------------------
// Library-owned scratch for ttm_chain_noalloc: a fixed device array in this
// code object, one copy per GPU, held until the process ends.  Host code
// never uses the array's name as an address (on the host it names a
// stand-in); the device address comes from hipGetSymbolAddress, taken once
// per device with that device current and kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TTM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

static int noalloc_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TTM_ERR_HIP;
    if (dev < 0 || dev >= 64) return TTM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TTM_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TTM_OK;
}

}  // namespace ttm

using namespace ttm;

extern "C" {

int ttm_chain_supported(int x, int f, int y, int m) { return combo_ok(x, f, y, m) ? 1 : 0; }

size_t ttm_chain_workspace_size(const ttm_shape *s, int x_dtype, int math) {
    if (validate_shape(s) != TTM_OK) return 0;
    const int f = math == TTM_MATH_F64 ? TTM_F64 : TTM_F32;
    if (!combo_ok(x_dtype, f, f, math)) return 0;
    ChainPlan p;
    if (!make_plan(*s, x_dtype, math, p)) return 0;
    return p.total;
}

int ttm_chain(const ttm_shape *s, const void *X, int x_dtype, const void *A, const void *B, const void *C,
              int f_dtype, void *Y, int y_dtype, int math, void *ws, size_t ws_bytes, void *stream) {
    ChainPlan p;
    int rc = chain_check(s, X, x_dtype, A, B, C, f_dtype, Y, y_dtype, math, p);
    if (rc) return rc;
    return chain_run(p, s, X, A, B, C, Y, math, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int ttm_chain_noalloc(const ttm_shape *s, const void *X, int x_dtype, const void *A, const void *B,
                      const void *C, int f_dtype, void *Y, int y_dtype, int math, void *stream) {
    ChainPlan p;
    int rc = chain_check(s, X, x_dtype, A, B, C, f_dtype, Y, y_dtype, math, p);
    if (rc) return rc;
    if (p.total > TTM_NOALLOC_SCRATCH_BYTES) return TTM_ERR_WORKSPACE;
    void *ws = nullptr;
    rc = noalloc_scratch(&ws);
    if (rc) return rc;
    return chain_run(p, s, X, A, B, C, Y, math, ws, TTM_NOALLOC_SCRATCH_BYTES, static_cast<hipStream_t>(stream));
}

}  // extern "C"
