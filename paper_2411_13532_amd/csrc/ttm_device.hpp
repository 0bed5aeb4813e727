// ttm_device.hpp -- device-side building blocks shared by the libttm kernels
// (gfx950, wave64): number formats, the bfloat16 split, and the matrix-core
// (MFMA) fragment conventions every contraction kernel uses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttm {

enum Math { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_BF16X3 = 3 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// bfloat16 is carried as its 16-bit pattern (the upper half of a float).
struct bf16_t { uint16_t bits; };

// float -> bfloat16 conversions use the gfx950 converter (v_cvt_pk_bf16_f32),
// which rounds to nearest with ties to even (the default rounding mode) and
// keeps NaN a NaN; two values per instruction, first value in the low half.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b) {
    bf16x2_t v = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint32_t bf16_rne_bits(float f) { return cvt_pk_bf16(f, 0.f) & 0xffffu; }
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// v = hi + lo + r with hi = rne(v), lo = rne(v - hi); v - hi is exact in float.
__device__ __forceinline__ void bf16_split(float v, uint32_t &hi, uint32_t &lo) {
    hi = bf16_rne_bits(v);
    lo = bf16_rne_bits(v - bf16_bits_to_f32(hi));
}
// The same for a pair (a in the low half): packed hi and packed lo.
__device__ __forceinline__ void bf16_split2(float a, float b, uint32_t &hi, uint32_t &lo) {
    hi = cvt_pk_bf16(a, b);
    lo = cvt_pk_bf16(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}
// Eight floats -> 8 packed bf16 (hi) and, when lo != nullptr, the residuals.
__device__ __forceinline__ void bf16_split8(const float (&v)[8], u32x4 &hi, u32x4 *lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bf16_split2(v[2 * i], v[2 * i + 1], h[i], l[i]);
    hi = u32x4{h[0], h[1], h[2], h[3]};
    if (lo) *lo = u32x4{l[0], l[1], l[2], l[3]};
}
__device__ __forceinline__ u32x4 bf16_round8(const float (&v)[8]) {
    return u32x4{cvt_pk_bf16(v[0], v[1]), cvt_pk_bf16(v[2], v[3]), cvt_pk_bf16(v[4], v[5]), cvt_pk_bf16(v[6], v[7])};
}

__device__ __forceinline__ uint32_t pack2(uint32_t a, uint32_t b) { return a | (b << 16); }

// ---------------------------------------------------------------------------
// MFMA 16x16 fragment conventions (wave64).
//
// For every 16x16 tile shape used here (f64 16x16x4, f32 16x16x4, bf16
// 16x16x32) a lane l owns row/column (l % 16) of the A/B operand and k-slot
// group g = l / 16.  Accumulator register r of lane l holds D[row][l % 16]
// with row = 4*g + r for the f32-accumulating shapes and row = 4*r + g for
// f64 16x16x4 (acc_row below); both layouts were checked on gfx950 with
// integer-valued operands.  Which k value a (group, element) slot carries is our choice as
// long as the A and B operands agree, so a lane always holds k values that are
// contiguous in memory: one 16-byte load feeds the operand of
//   bf16: 1 MFMA (8 values),  f32: 4 MFMAs (4 values),  f64: 2 MFMAs (2 values).
// A "k-group" is the 4 * (values per 16 bytes) k indices one such load covers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int MATH> struct MathTraits;
template <> struct MathTraits<M_F64> {
    typedef double acc_t; typedef f64x4 accv_t; typedef double fac_t;   // factor storage
    typedef double lds_t;                                                // operand storage
    static constexpr int VE = 2;            // values per 16 bytes of operand
    static constexpr int KG = 4 * VE;       // k indices per k-group
    __device__ static constexpr int acc_row(int g, int r) { return 4 * r + g; }
};
template <> struct MathTraits<M_F32> {
    typedef float acc_t; typedef f32x4 accv_t; typedef float fac_t; typedef float lds_t;
    static constexpr int VE = 4;
    static constexpr int KG = 4 * VE;
    __device__ static constexpr int acc_row(int g, int r) { return 4 * g + r; }
};
template <> struct MathTraits<M_BF16> {
    typedef float acc_t; typedef f32x4 accv_t; typedef uint16_t fac_t; typedef uint16_t lds_t;
    static constexpr int VE = 8;
    static constexpr int KG = 4 * VE;
    __device__ static constexpr int acc_row(int g, int r) { return 4 * g + r; }
};
template <> struct MathTraits<M_BF16X3> : MathTraits<M_BF16> {};

template <typename T> __device__ __forceinline__ T zero_accv();
template <> __device__ __forceinline__ f32x4 zero_accv<f32x4>() { return f32x4{0.f, 0.f, 0.f, 0.f}; }
template <> __device__ __forceinline__ f64x4 zero_accv<f64x4>() { return f64x4{0.0, 0.0, 0.0, 0.0}; }

// 16-byte register vector, reinterpretable as 4 floats, 2 doubles or 8 bf16.
union V16 {
    u32x4 u;
    float f[4];
    double d[2];
    uint16_t h[8];
};

__device__ __forceinline__ V16 ld16(const void *p) {
    V16 v;
    v.u = *reinterpret_cast<const u32x4 *>(p);
    return v;
}
__device__ __forceinline__ V16 zero16() {
    V16 v;
    v.u = u32x4{0u, 0u, 0u, 0u};
    return v;
}

// One matrix-core step for a k-group: A and B hold one 16-byte operand
// fragment each (row/col l%16, values of k-slot group l/16).  For bf16x3 the
// optional lo fragments add the cross terms hi*lo' + lo*hi'.
template <int MATH>
__device__ __forceinline__ void mma_kgroup(typename MathTraits<MATH>::accv_t &acc, const V16 &a, const V16 &b);

template <>
__device__ __forceinline__ void mma_kgroup<M_F64>(f64x4 &acc, const V16 &a, const V16 &b) {
    acc = mfma_f64(a.d[0], b.d[0], acc);
    acc = mfma_f64(a.d[1], b.d[1], acc);
}
template <>
__device__ __forceinline__ void mma_kgroup<M_F32>(f32x4 &acc, const V16 &a, const V16 &b) {
    acc = mfma_f32(a.f[0], b.f[0], acc);
    acc = mfma_f32(a.f[1], b.f[1], acc);
    acc = mfma_f32(a.f[2], b.f[2], acc);
    acc = mfma_f32(a.f[3], b.f[3], acc);
}
template <>
__device__ __forceinline__ void mma_kgroup<M_BF16>(f32x4 &acc, const V16 &a, const V16 &b) {
    acc = mfma_bf16(a.u, b.u, acc);
}

// 16 bytes per lane from global memory straight into LDS (global_load_lds,
// gfx950): lane l of the wave writes lds_wave_base + 16*l.  `lds_wave_base`
// must be the same for the whole wave.  The builtin exists only in the device
// compilation; the host pass sees an empty body.
__device__ __forceinline__ void dma16_to_lds(const void *g, void *lds_wave_base) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(const_cast<void *>(g), lds_wave_base, 16, 0, 0);
#endif
}

__device__ __forceinline__ uint32_t lds_offset(const void *p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char *)p));
}
// Direct-to-LDS copy of 16 bytes per lane to LDS byte address m0 + 16 lane,
// issued through inline assembly so that the compiler does not count it among
// the vector-memory operations it waits for: its own waits for ordinary loads
// (which return in order among themselves) then count only those loads
// instead of falling back to waiting for everything, and the copies are waited
// for explicitly (wait_vmcnt).  The LDS address is bound to m0 through the
// operand constraint, so the compiler writes m0 itself and knows it is taken;
// the s_nop separates that write from the copy that reads it.
__device__ __forceinline__ void dma16_to_lds_m0(const void *g, uint32_t lds_addr) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(g), "{m0}"(lds_addr) : "memory");
}
// The same with a wave-uniform base in SGPRs and a 32-bit per-lane byte
// offset (below 2^31): the lane's address is sbase + voff, formed by the
// memory unit, so the lane holds one register instead of a 64-bit address.
__device__ __forceinline__ void dma16s_to_lds_m0(const void *sbase, uint32_t voff, uint32_t lds_addr) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" : : "v"(voff), "s"(sbase), "{m0}"(lds_addr) : "memory");
}
// The same for 4 bytes per lane (LDS byte address m0 + 4 lane).
__device__ __forceinline__ void dma4_to_lds_m0(const void *g, uint32_t lds_addr) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, off" : : "v"(g), "{m0}"(lds_addr) : "memory");
}
// wait until at most N vector-memory operations of this wave are outstanding
// (they complete in issue order)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xf) | ((N >> 4) << 14) | (0x7 << 4) | (0xf << 8));
}

// LDS accesses of one wavefront are performed in issue order; this only stops
// the compiler from moving them across a point where the wave's lanes hand
// data to each other through LDS.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Host/device rounding helpers for sizes.
__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace ttm
