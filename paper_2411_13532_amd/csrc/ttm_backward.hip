// ttm_backward.hip -- adjoint of the chain Y = X x1 A x2 B x3 C.
//
// Given G = dL/dY (J1 x J2 x J3), every gradient is a contraction of G
// with the inputs, evaluated as a short sequence of unfolded products on
// the matrix cores (k_gemm), each reading its operands in place:
//   W  = X x3 C                 (I1 I2 x J3)      = X_(12) C^T
//   V  = W x2 B = X x2 B x3 C   (I1 x J2 x J3)    per i1: B W[i1]
//   H  = G x1 A^T               (I1 x J2 x J3)    = A^T G_(1)
//   R  = H x2 B^T               (I1 x I2 x J3)    per i1: B^T H[i1]
//   dX = R x3 C^T               (I1 x I2 x I3)    = R_(12) C
//   dA = G_(1) V_(1)^T          (J1 x I1)
//   dB = sum_{i1,j3} H[i1,j2,j3] W[i1,i2,j3]       (J2 x I2)
//   dC = R_(3) X_(3)^T          (J3 x I3)
// so dX = G x1 A^T x2 B^T x3 C^T and each factor gradient contracts G with
// the input chain that skips that factor.  Long contractions (over I1*I2 or
// I1*J3) are split over workgroups and summed in a fixed order.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "ttm_gemm.hpp"
#include "ttm_host.hpp"

namespace ttm {

namespace {

struct BwdPlan {
    int math;
    size_t esz;
    int64_t I1, I2, I3, J1, J2, J3, NN;
    bool need_w, need_v, need_h, need_r;
    size_t off_W, off_V, off_H, off_R, off_P, total;
    int64_t part_elems;
    // float32 with J3 <= 32 (a multiple of 4) and I3 a multiple of 64: the
    // X-sized products (W, dX, dC) run on the streaming kernels below
    bool skinny;
    bool skinny_vr;   // also J2 <= 32 and I2 a multiple of 64: V and R on streaming kernels
    int dc_splits;
    int64_t dc_rows;
};

constexpr int64_t KT_F32 = 32, KT_F64 = 16;
// partials per group of the first stage of the two-level split sums
constexpr int SUM_GROUP = 16;

struct SplitK {
    int ks;
    int64_t per;
};

SplitK choose_split(int64_t M, int64_t N, int64_t K, int64_t batch, int64_t KT) {
    const int64_t tiles = ceil_div(M, 64) * ceil_div(N, 64) * batch;
    int64_t ks = ceil_div(512, tiles);
    ks = std::max<int64_t>(1, std::min<int64_t>(ks, ceil_div(K, KT * 4)));
    ks = std::min<int64_t>(ks, 256);
    const int64_t per = round_up(ceil_div(K, ks), KT);
    return {int(ceil_div(K, per)), per};
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

void make_bwd_plan(const ttm_shape &s, int math, bool dX, bool dA, bool dB, bool dC, BwdPlan &p) {
    p = BwdPlan();
    p.math = math;
    p.esz = math == TTM_MATH_F64 ? 8 : 4;
    p.I1 = s.I[0]; p.I2 = s.I[1]; p.I3 = s.I[2];
    p.J1 = s.J[0]; p.J2 = s.J[1]; p.J3 = s.J[2];
    p.NN = p.J2 * p.J3;
    p.need_w = dA || dB;
    p.need_v = dA;
    p.need_h = dX || dB || dC;
    p.need_r = dX || dC;
    const int64_t KT = math == TTM_MATH_F64 ? KT_F64 : KT_F32;
    // partial buffers of the split contractions
    p.part_elems = 0;
    // partials of a split, then (more than SUM_GROUP of them) their group sums
    auto split_elems = [](int ks, int64_t mn) { return (int64_t(ks) + (ks > SUM_GROUP ? ceil_div(ks, SUM_GROUP) : 0)) * mn; };
    if (dA) {
        SplitK k = choose_split(p.J1, p.I1, p.NN, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, split_elems(k.ks, p.J1 * p.I1));
    }
    if (dB) {
        SplitK k = choose_split(p.J2, p.I2, p.I1 * p.J3, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, split_elems(k.ks, p.J2 * p.I2));
    }
    const int64_t M = p.I1 * p.I2;
    p.skinny = math == TTM_MATH_F32 && p.J3 <= 32 && p.J3 % 4 == 0 && p.I3 % 64 == 0 && M < (int64_t(1) << 31) &&
               p.I3 < (int64_t(1) << 24);
    p.skinny_vr = p.skinny && p.J2 <= 32 && p.I2 % 64 == 0 && p.I2 < (int64_t(1) << 24) && p.I1 < (int64_t(1) << 31);
    if (dC) {
        SplitK k = choose_split(p.J3, p.I3, p.I1 * p.I2, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, split_elems(k.ks, p.J3 * p.I3));
        if (p.skinny) {
            const int64_t s0 = std::min<int64_t>(512, ceil_div(M, 64));
            p.dc_rows = round_up(ceil_div(M, s0), 4);
            p.dc_splits = int(ceil_div(M, p.dc_rows));
            // the partials, then their group sums
            p.part_elems =
                std::max(p.part_elems, (int64_t(p.dc_splits) + ceil_div(p.dc_splits, SUM_GROUP)) * p.J3 * p.I3);
        }
    }
    size_t off = 0;
    auto take = [&](bool need, int64_t elems) -> size_t {
        if (!need) return 0;
        size_t o = off;
        off = al256(off + size_t(elems) * p.esz);
        return o;
    };
    p.off_W = take(p.need_w, p.I1 * p.I2 * p.J3);
    p.off_V = take(p.need_v, p.I1 * p.NN);
    p.off_H = take(p.need_h, p.I1 * p.NN);
    p.off_R = take(p.need_r, p.I1 * p.I2 * p.J3);
    p.off_P = take(p.part_elems > 0, p.part_elems);
    p.total = off;
}

GemmArgs gargs() {
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.P = 1;
    return a;
}

// ---------------------------------------------------------------------------
// Streaming kernels for the three products of the adjoint that read or write
// an X-sized tensor, in float32 with J3 <= 32 (a multiple of 4) and I3 a
// multiple of 64.  Rows r = (i1, i2) of X, dX (I3 long) and of W, R (J3 long).
// Each lane reads 16 bytes of the X-sized operand (or writes them, for dX)
// straight into a 16 x 16 x 4 matrix-core operand: which k (or n) value a
// (lane group, element) slot carries is free as long as both operands agree,
// so one 16-byte access feeds four products.  No LDS, no barriers; the small
// operands (C, R) come through the caches.
// ---------------------------------------------------------------------------
constexpr int SK_WAVES = 4;

// W[r][j] = sum_k X[r][k] C[j][k].  A wave owns 32 rows (two 16-row blocks)
// and all 32 columns; k slot (g, s) of chunk k0 carries k = k0 + 4 g + s.
__global__ void __launch_bounds__(64 * SK_WAVES) k_bwd_w_f32(const float *__restrict__ X, const float *__restrict__ C,
                                                            float *__restrict__ W, int64_t M, int I3, int J3) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int64_t r0 = (int64_t(blockIdx.x) * SK_WAVES + wave) * 32;
    if (r0 >= M) return;
    const float *xr[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int64_t row = r0 + mb * 16 + l16;
        xr[mb] = X + (row < M ? row : M - 1) * I3 + 4 * g;
    }
    const bool cv[2] = {l16 < J3, 16 + l16 < J3};
    const float *cr[2] = {C + int64_t(cv[0] ? l16 : 0) * I3 + 4 * g, C + int64_t(cv[1] ? 16 + l16 : 0) * I3 + 4 * g};
    f32x4 acc[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = zero_accv<f32x4>();
    for (int k0 = 0; k0 < I3; k0 += 64) {
        V16 xa[2][4], cb[2][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) xa[mb][u] = ld16(xr[mb] + k0 + 16 * u);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                cb[nb][u] = ld16(cr[nb] + k0 + 16 * u);
                if (!cv[nb]) cb[nb][u] = zero16();
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = mfma_f32(xa[mb][u].f[e], cb[nb][u].f[e], acc[mb][nb]);
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t row = r0 + mb * 16 + 4 * g + rr;
            if (row >= M) continue;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                if (cv[nb]) W[row * J3 + nb * 16 + l16] = acc[mb][nb][rr];
        }
}

// part[s][j][i] = sum_{r in split s} R[r][j] X[r][i].  grid (splits,
// ceil(I3 / 256)); a wave owns 64 columns i; k slot g of a step carries row
// r0 + g, and column n of product e is i = i0 + 4 n + e.
__global__ void __launch_bounds__(64 * SK_WAVES) k_bwd_dc_f32(const float *__restrict__ R, const float *__restrict__ X,
                                                             float *__restrict__ part, int64_t M, int I3, int J3,
                                                             int64_t rows_per_split) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int i0 = (blockIdx.y * SK_WAVES + wave) * 64;
    if (i0 >= I3) return;
    const int64_t rb = int64_t(blockIdx.x) * rows_per_split;
    const int64_t re = M < rb + rows_per_split ? M : rb + rows_per_split;
    const bool jv[2] = {l16 < J3, 16 + l16 < J3};
    f32x4 acc[2][4];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[jb][e] = zero_accv<f32x4>();
    for (int64_t r0 = rb; r0 < re; r0 += 16) {
        V16 xb[4];
        float ra[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = r0 + 4 * u + g;
            const bool ok = row < re;
            const int64_t rc = ok ? row : rb;
            xb[u] = ld16(X + rc * I3 + i0 + 4 * l16);
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                const float v = R[rc * J3 + (jv[jb] ? jb * 16 + l16 : 0)];
                ra[u][jb] = ok && jv[jb] ? v : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb) acc[jb][e] = mfma_f32(ra[u][jb], xb[u].f[e], acc[jb][e]);
    }
    float *pp = part + int64_t(blockIdx.x) * J3 * I3;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int j = jb * 16 + 4 * g + rr;
            if (j >= J3) continue;
            const f32x4 v = {acc[jb][0][rr], acc[jb][1][rr], acc[jb][2][rr], acc[jb][3][rr]};
            *reinterpret_cast<f32x4 *>(pp + int64_t(j) * I3 + i0 + 4 * l16) = v;
        }
}

// dX[r][i] = sum_j R[r][j] C[j][i].  grid (ceil(M / DX_ROWS), ceil(I3 /
// 256)); a wave owns 64 columns i and keeps their C fragments in
// registers; k slot (g, e) of half h carries j = 16 h + 4 g + e, column n of
// output product t is i = i0 + 4 n + t, so each lane stores 16 bytes per row.
constexpr int DX_ROWS = 64;
__global__ void __launch_bounds__(64 * SK_WAVES) k_bwd_dx_f32(const float *__restrict__ R, const float *__restrict__ C,
                                                             float *__restrict__ dX, int64_t M, int I3, int J3) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int i0 = (blockIdx.y * SK_WAVES + wave) * 64;
    if (i0 >= I3) return;
    const int64_t rb = int64_t(blockIdx.x) * DX_ROWS;
    const int64_t re = M < rb + DX_ROWS ? M : rb + DX_ROWS;
    V16 cf[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 16 * h + 4 * g + e;
            cf[h][e] = ld16(C + int64_t(j < J3 ? j : 0) * I3 + i0 + 4 * l16);
            if (j >= J3) cf[h][e] = zero16();
        }
    const bool hv[2] = {4 * g < J3, 16 + 4 * g < J3};
    // the R fragments of all DX_ROWS rows are loaded first
    V16 ra[DX_ROWS / 16][2];
#pragma unroll
    for (int q = 0; q < DX_ROWS / 16; ++q) {
        const int64_t row = rb + 16 * q + l16;
        const int64_t rc = row < re ? row : re - 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            ra[q][h] = ld16(R + rc * J3 + (hv[h] ? 16 * h + 4 * g : 0));
            if (!hv[h]) ra[q][h] = zero16();
        }
    }
#pragma unroll
    for (int q = 0; q < DX_ROWS / 16; ++q) {
        const int64_t r0 = rb + 16 * q;
        if (r0 >= re) break;
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = zero_accv<f32x4>();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] = mfma_f32(ra[q][h].f[e], cf[h][e].f[t], acc[t]);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t r = r0 + 4 * g + rr;
            if (r >= re) continue;
            const f32x4 v = {acc[0][rr], acc[1][rr], acc[2][rr], acc[3][rr]};
            *reinterpret_cast<f32x4 *>(dX + r * I3 + i0 + 4 * l16) = v;
        }
    }
}

// V[i1][j2][j3] = sum_i2 B[j2][i2] W[i1][i2][j3] (J2, J3 <= 32, I2 a
// multiple of 64).  A workgroup owns one i1; its four waves split the i2
// range into quarters and add their 32 x 32 partials through LDS in a fixed
// order.  k slot (g, e) of chunk k0 carries i2 = k0 + 4 g + e: B is read 16
// bytes per lane, W one float per lane (16 consecutive j3 of a row).
__global__ void __launch_bounds__(64 * SK_WAVES) k_bwd_v_f32(const float *__restrict__ B, const float *__restrict__ W,
                                                            float *__restrict__ V, int64_t I1, int I2, int J2,
                                                            int J3) {
    __shared__ float red[SK_WAVES - 1][32 * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int64_t i1 = blockIdx.x;
    const int q = I2 / SK_WAVES, kb = wave * q;
    const bool bv[2] = {l16 < J2, 16 + l16 < J2}, wv[2] = {l16 < J3, 16 + l16 < J3};
    const float *brow[2] = {B + int64_t(bv[0] ? l16 : 0) * I2 + 4 * g, B + int64_t(bv[1] ? 16 + l16 : 0) * I2 + 4 * g};
    const float *wcol[2] = {W + i1 * I2 * J3 + (wv[0] ? l16 : 0), W + i1 * I2 * J3 + (wv[1] ? 16 + l16 : 0)};
    f32x4 acc[2][2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[jb][nb] = zero_accv<f32x4>();
    for (int k0 = kb; k0 < kb + q; k0 += 16) {
        V16 ba[2];
        float wb[2][4];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            ba[jb] = ld16(brow[jb] + k0);
            if (!bv[jb]) ba[jb] = zero16();
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float x = wcol[nb][int64_t(k0 + 4 * g + e) * J3];
                wb[nb][e] = wv[nb] ? x : 0.f;
            }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) acc[jb][nb] = mfma_f32(ba[jb].f[e], wb[nb][e], acc[jb][nb]);
    }
    // element (jb, nb, rr) of a lane: j2 = 16 jb + 4 g + rr, j3 = 16 nb + l16
    if (wave > 0) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) red[wave - 1][((jb * 2 + nb) * 4 + rr) * 64 + lane] = acc[jb][nb][rr];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < SK_WAVES - 1; ++w)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) acc[jb][nb][rr] += red[w][((jb * 2 + nb) * 4 + rr) * 64 + lane];
    float *Vp = V + i1 * J2 * J3;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int j2 = 16 * jb + 4 * g + rr;
            if (j2 >= J2) continue;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                if (wv[nb]) Vp[j2 * J3 + 16 * nb + l16] = acc[jb][nb][rr];
        }
}

// R[i1][i2][j3] = sum_j2 B[j2][i2] H[i1][j2][j3] (J2, J3 <= 32).  A wave owns
// 64 rows i2 of one i1 (grid (I1, ceil(I2 / 256))); k slot g of step s
// carries j2 = 4 s + g; B and H are read one float per lane (16 consecutive
// i2 or j3), R written 64 contiguous bytes per row and 16 lanes.
__global__ void __launch_bounds__(64 * SK_WAVES) k_bwd_r_f32(const float *__restrict__ B, const float *__restrict__ H,
                                                            float *__restrict__ R, int64_t I1, int I2, int J2,
                                                            int J3) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int64_t i1 = blockIdx.x;
    const int m0 = (blockIdx.y * SK_WAVES + wave) * 64;
    if (m0 >= I2) return;
    const bool nv[2] = {l16 < J3, 16 + l16 < J3};
    const float *Hp = H + i1 * J2 * J3;
    f32x4 acc[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = zero_accv<f32x4>();
    for (int s = 0; 4 * s < J2; ++s) {
        const int j2 = 4 * s + g;
        const bool kv = j2 < J2;
        const int j2c = kv ? j2 : 0;
        float a[4], h[2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int i2 = m0 + 16 * mb + l16;
            const float x = B[int64_t(j2c) * I2 + (i2 < I2 ? i2 : I2 - 1)];
            a[mb] = kv && i2 < I2 ? x : 0.f;
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const float x = Hp[j2c * J3 + (nv[nb] ? 16 * nb + l16 : 0)];
            h[nb] = kv && nv[nb] ? x : 0.f;
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = mfma_f32(a[mb], h[nb], acc[mb][nb]);
    }
    float *Rp = R + i1 * int64_t(I2) * J3;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i2 = m0 + 16 * mb + 4 * g + rr;
            if (i2 >= I2) continue;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                if (nv[nb]) Rp[int64_t(i2) * J3 + 16 * nb + l16] = acc[mb][nb][rr];
        }
}

// First stage of a two-level fixed-order sum of S partials of n elements:
// out[b][e] = sum_{s < G, b G + s < S} part[(b G + s) * n + e], increasing s;
// grid (ceil(n / 256), ceil(S / G)).
__global__ void __launch_bounds__(256) k_sum_groups_f32(const float *__restrict__ part, int64_t n, int S,
                                                       float *__restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= n) return;
    const int s0 = blockIdx.y * SUM_GROUP;
    const int cnt = S - s0 < SUM_GROUP ? S - s0 : SUM_GROUP;
    float v[SUM_GROUP];
#pragma unroll
    for (int s = 0; s < SUM_GROUP; ++s) {
        const float x = part[int64_t(s0 + (s < cnt ? s : 0)) * n + e];
        v[s] = s < cnt ? x : 0.f;
    }
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < SUM_GROUP; ++s) acc += v[s];
    out[int64_t(blockIdx.y) * n + e] = acc;
}

template <int MATH>
int run_gemm(GemmArgs a, int64_t batch, bool split, void *part, hipStream_t st, const char *name) {
    typedef typename MathTraits<MATH>::acc_t T;
    const int64_t KT = GemmCfg<MATH>::KT;
    if (a.Ki <= 0) a.Ki = a.K;
    SplitK k = split ? choose_split(a.M, a.N, a.K, batch, KT) : SplitK{1, round_up(a.K, KT)};
    void *final_out = a.C;
    if (k.ks > 1) {
        // partials are dense row-major M x N (batch must be 1 here)
        a.C = part;
        a.scm = a.N;
        a.scn = 1;
        a.scs = a.M * a.N;
    }
    a.k_per_split = k.per;
    // 16-byte operand loads along the unit-stride dimension where every
    // group of VG elements stays inside the extent, the k split and one
    // address-aligned run
    {
        const int64_t VG = int64_t(16 / sizeof(T));
        const bool kk = a.K % VG == 0 && a.Ki % VG == 0 && a.k_per_split % VG == 0;
        auto vec_ok = [&](const void *ptr, int64_t sfast_m, int64_t sk, int64_t sko, int64_t sb, int64_t sp,
                          int64_t extent) -> int {
            if (!aligned(ptr, 16) || sb % VG || sp % VG) return 0;
            if (sk == 1) return (kk && sfast_m % VG == 0 && (a.Ki == a.K || sko % VG == 0)) ? 1 : 0;
            if (sfast_m == 1) return (extent % VG == 0 && sk % VG == 0 && (a.Ki == a.K || sko % VG == 0)) ? 1 : 0;
            return 0;
        };
        a.vec_a = vec_ok(a.A, a.sam, a.saki, a.sako, a.sab, 0, a.M);
        a.vec_b = vec_ok(a.B, a.sbn, a.sbki, a.sbko, a.sbb, a.P > 1 ? a.sbp : 0, a.N);
    }
    dim3 grid(unsigned(ceil_div(a.M, 64) * ceil_div(a.N, 64)), unsigned(k.ks), unsigned(batch));
    int rc = launch(name, st, [&] {
        if (a.vec_a && a.vec_b) hipLaunchKernelGGL((k_gemm<MATH, true, true>), grid, dim3(256), 0, st, a);
        else if (a.vec_a) hipLaunchKernelGGL((k_gemm<MATH, true, false>), grid, dim3(256), 0, st, a);
        else if (a.vec_b) hipLaunchKernelGGL((k_gemm<MATH, false, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gemm<MATH, false, false>), grid, dim3(256), 0, st, a);
    });
    if (rc || k.ks == 1) return rc;
    const int64_t n = a.M * a.N;
    dim3 rg(unsigned(std::min<int64_t>(ceil_div(n, 256), 4096)));
    if constexpr (std::is_same<T, float>::value) {
        if (k.ks > SUM_GROUP) {   // groups of SUM_GROUP partials, then the group sums, in order
            const int ng = int(ceil_div(k.ks, SUM_GROUP));
            T *pg = static_cast<T *>(part) + int64_t(k.ks) * n;
            rc = launch("ttm_bwd_sum_splits", st, [&] {
                hipLaunchKernelGGL(k_sum_groups_f32, dim3(unsigned(ceil_div(n, 256)), unsigned(ng)), dim3(256), 0, st,
                                   static_cast<const float *>(part), n, k.ks, pg);
            });
            if (rc) return rc;
            return launch("ttm_bwd_sum_splits", st, [&] {
                hipLaunchKernelGGL(k_sum_splits<T>, rg, dim3(256), 0, st, static_cast<const T *>(pg), n, ng, n,
                                   static_cast<T *>(final_out));
            });
        }
    }
    return launch("ttm_bwd_sum_splits", st, [&] {
        hipLaunchKernelGGL(k_sum_splits<T>, rg, dim3(256), 0, st, static_cast<const T *>(part), a.M * a.N, k.ks, n,
                           static_cast<T *>(final_out));
    });
}

template <int MATH>
int run_backward(const BwdPlan &p, const void *G, const void *X, const void *A, const void *B, const void *C,
                 void *dX, void *dA, void *dB, void *dC, unsigned char *ws, hipStream_t st) {
    void *W = ws + p.off_W, *V = ws + p.off_V, *H = ws + p.off_H, *R = ws + p.off_R, *Pt = ws + p.off_P;
    const int64_t I1 = p.I1, I2 = p.I2, I3 = p.I3, J1 = p.J1, J2 = p.J2, J3 = p.J3, NN = p.NN;
    // the streaming kernels read X and C 16 bytes at a time
    const bool skinny = p.skinny && aligned(X, 16) && aligned(C, 16);
    int rc = TTM_OK;
    if (p.need_w) {   // W[(i1,i2)][j3] = sum_i3 X[(i1,i2)][i3] C[j3][i3]
        GemmArgs a = gargs();
        a.A = X; a.B = C; a.C = W;
        a.M = I1 * I2; a.N = J3; a.K = I3;
        a.sam = I3; a.saki = 1;
        a.sbn = I3; a.sbki = 1;
        a.scm = J3; a.scn = 1;
        if (MATH == M_F32 && skinny) {
            const int64_t M = I1 * I2;
            rc = launch("ttm_bwd_W", st, [&] {
                hipLaunchKernelGGL(k_bwd_w_f32, dim3(unsigned(ceil_div(M, 32 * SK_WAVES))), dim3(64 * SK_WAVES), 0, st,
                                   static_cast<const float *>(X), static_cast<const float *>(C), static_cast<float *>(W),
                                   M, int(I3), int(J3));
            });
            if (rc) return rc;
        } else if ((rc = run_gemm<MATH>(a, 1, false, nullptr, st, "ttm_bwd_W"))) {
            return rc;
        }
    }
    if (p.need_v) {   // V[i1][j2][j3] = sum_i2 B[j2][i2] W[i1][i2][j3]
        GemmArgs a = gargs();
        a.A = B; a.B = W; a.C = V;
        a.M = J2; a.N = J3; a.K = I2;
        a.sam = I2; a.saki = 1;
        a.sbb = I2 * J3; a.sbki = J3; a.sbn = 1;
        a.scb = NN; a.scm = J3; a.scn = 1;
        if (MATH == M_F32 && p.skinny_vr && aligned(B, 16)) {
            rc = launch("ttm_bwd_V", st, [&] {
                hipLaunchKernelGGL(k_bwd_v_f32, dim3(unsigned(I1)), dim3(64 * SK_WAVES), 0, st,
                                   static_cast<const float *>(B), static_cast<const float *>(W), static_cast<float *>(V),
                                   I1, int(I2), int(J2), int(J3));
            });
            if (rc) return rc;
        } else if ((rc = run_gemm<MATH>(a, I1, false, nullptr, st, "ttm_bwd_V"))) {
            return rc;
        }
    }
    if (dA) {         // dA[j1][i1] = sum_n G[j1][n] V[i1][n]
        GemmArgs a = gargs();
        a.A = G; a.B = V; a.C = dA;
        a.M = J1; a.N = I1; a.K = NN;
        a.sam = NN; a.saki = 1;
        a.sbn = NN; a.sbki = 1;
        a.scm = I1; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, 1, true, Pt, st, "ttm_bwd_dA"))) return rc;
    }
    if (p.need_h) {   // H[i1][n] = sum_j1 A[j1][i1] G[j1][n]
        GemmArgs a = gargs();
        a.A = A; a.B = G; a.C = H;
        a.M = I1; a.N = NN; a.K = J1;
        a.sam = 1; a.saki = I1;
        a.sbn = 1; a.sbki = NN;
        a.scm = NN; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, 1, false, nullptr, st, "ttm_bwd_H"))) return rc;
    }
    if (p.need_r) {   // R[i1][i2][j3] = sum_j2 B[j2][i2] H[i1][j2][j3]
        GemmArgs a = gargs();
        a.A = B; a.B = H; a.C = R;
        a.M = I2; a.N = J3; a.K = J2;
        a.sam = 1; a.saki = I2;
        a.sbb = NN; a.sbki = J3; a.sbn = 1;
        a.scb = I2 * J3; a.scm = J3; a.scn = 1;
        if (MATH == M_F32 && p.skinny_vr) {
            rc = launch("ttm_bwd_R", st, [&] {
                hipLaunchKernelGGL(k_bwd_r_f32, dim3(unsigned(I1), unsigned(ceil_div(I2, 64 * SK_WAVES))),
                                   dim3(64 * SK_WAVES), 0, st, static_cast<const float *>(B),
                                   static_cast<const float *>(H), static_cast<float *>(R), I1, int(I2), int(J2),
                                   int(J3));
            });
            if (rc) return rc;
        } else if ((rc = run_gemm<MATH>(a, I1, false, nullptr, st, "ttm_bwd_R"))) {
            return rc;
        }
    }
    if (dX) {         // dX[(i1,i2)][i3] = sum_j3 R[(i1,i2)][j3] C[j3][i3]
        GemmArgs a = gargs();
        a.A = R; a.B = C; a.C = dX;
        a.M = I1 * I2; a.N = I3; a.K = J3;
        a.sam = J3; a.saki = 1;
        a.sbn = 1; a.sbki = I3;
        a.scm = I3; a.scn = 1;
        if (MATH == M_F32 && skinny && aligned(dX, 16)) {
            const int64_t M = I1 * I2;
            rc = launch("ttm_bwd_dX", st, [&] {
                hipLaunchKernelGGL(k_bwd_dx_f32, dim3(unsigned(ceil_div(M, DX_ROWS)), unsigned(ceil_div(I3, 64 * SK_WAVES))),
                                   dim3(64 * SK_WAVES), 0, st, static_cast<const float *>(R),
                                   static_cast<const float *>(C), static_cast<float *>(dX), M, int(I3), int(J3));
            });
            if (rc) return rc;
        } else if ((rc = run_gemm<MATH>(a, 1, false, nullptr, st, "ttm_bwd_dX"))) {
            return rc;
        }
    }
    if (dB) {         // dB[j2][i2] = sum_{i1,j3} H[i1][j2][j3] W[i1][i2][j3]
        GemmArgs a = gargs();
        a.A = H; a.B = W; a.C = dB;
        a.M = J2; a.N = I2; a.K = I1 * J3; a.Ki = J3;
        a.sam = J3; a.sako = NN; a.saki = 1;
        a.sbn = J3; a.sbko = I2 * J3; a.sbki = 1;
        a.scm = I2; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, 1, true, Pt, st, "ttm_bwd_dB"))) return rc;
    }
    if (dC) {         // dC[j3][i3] = sum_{(i1,i2)} R[(i1,i2)][j3] X[(i1,i2)][i3]
        GemmArgs a = gargs();
        a.A = R; a.B = X; a.C = dC;
        a.M = J3; a.N = I3; a.K = I1 * I2;
        a.sam = 1; a.saki = J3;
        a.sbn = 1; a.sbki = I3;
        a.scm = I3; a.scn = 1;
        if (MATH == M_F32 && skinny) {
            const int64_t M = I1 * I2, n = J3 * I3;
            rc = launch("ttm_bwd_dC", st, [&] {
                hipLaunchKernelGGL(k_bwd_dc_f32, dim3(unsigned(p.dc_splits), unsigned(ceil_div(I3, 64 * SK_WAVES))),
                                   dim3(64 * SK_WAVES), 0, st, static_cast<const float *>(R),
                                   static_cast<const float *>(X), static_cast<float *>(Pt), M, int(I3), int(J3),
                                   p.dc_rows);
            });
            if (rc) return rc;
            // partials summed in groups of SUM_GROUP (in order), then the
            // group sums in order; the group sums go after the partials
            const int ng = int(ceil_div(p.dc_splits, SUM_GROUP));
            float *Pg = static_cast<float *>(Pt) + int64_t(p.dc_splits) * n;
            rc = launch("ttm_bwd_sum_splits", st, [&] {
                hipLaunchKernelGGL(k_sum_groups_f32, dim3(unsigned(ceil_div(n, 256)), unsigned(ng)), dim3(256), 0, st,
                                   static_cast<const float *>(Pt), n, p.dc_splits, Pg);
            });
            if (rc) return rc;
            dim3 rg(unsigned(std::min<int64_t>(ceil_div(n, 256), 4096)));
            rc = launch("ttm_bwd_sum_splits", st, [&] {
                hipLaunchKernelGGL(k_sum_splits<float>, rg, dim3(256), 0, st, static_cast<const float *>(Pg), n, ng,
                                   n, static_cast<float *>(dC));
            });
            if (rc) return rc;
        } else if ((rc = run_gemm<MATH>(a, 1, true, Pt, st, "ttm_bwd_dC"))) {
            return rc;
        }
    }
    return rc;
}

int validate(const ttm_shape *s) {
    if (!s) return TTM_ERR_INVALID_ARG;
    for (int n = 0; n < 3; ++n)
        if (s->I[n] < 1 || s->J[n] < 1 || s->I[n] > (int64_t(1) << 31) || s->J[n] > (int64_t(1) << 31))
            return TTM_ERR_INVALID_ARG;
    if (checked_prod(checked_prod(s->I[0], s->I[1]), s->I[2]) < 0) return TTM_ERR_INVALID_ARG;
    if (checked_prod(checked_prod(s->J[0], s->J[1]), s->J[2]) < 0) return TTM_ERR_INVALID_ARG;
    return TTM_OK;
}

bool bwd_combo_ok(int dtype, int math) {
    return (dtype == TTM_F64 && math == TTM_MATH_F64) || (dtype == TTM_F32 && math == TTM_MATH_F32);
}

}  // namespace
}  // namespace ttm

using namespace ttm;

extern "C" {

size_t ttm_chain_backward_workspace_size(const ttm_shape *s, int dtype, int math) {
    if (validate(s) != TTM_OK || !bwd_combo_ok(dtype, math)) return 0;
    BwdPlan p;
    make_bwd_plan(*s, math, true, true, true, true, p);
    return p.total;
}

int ttm_chain_backward(const ttm_shape *s, const void *G, const void *X, const void *A, const void *B, const void *C,
                       int dtype, void *dX, void *dA, void *dB, void *dC, int math, void *ws, size_t ws_bytes,
                       void *stream) {
    int rc = validate(s);
    if (rc) return rc;
    if (!bwd_combo_ok(dtype, math)) return TTM_ERR_UNSUPPORTED;
    // every contraction length must fit the GEMM's 32-bit k index
    const int64_t k_max = std::max({s->I[0] * s->I[1], s->I[0] * s->J[2], s->J[1] * s->J[2], s->I[1], s->I[2], s->J[0]});
    if (k_max >= (int64_t(1) << 32)) return TTM_ERR_UNSUPPORTED;
    if (!G || !X || !A || !B || !C) return TTM_ERR_INVALID_ARG;
    if (!dX && !dA && !dB && !dC) return TTM_ERR_INVALID_ARG;
    const size_t e = dtype_size(dtype);
    const void *ins[5] = {G, X, A, B, C};
    void *outs[4] = {dX, dA, dB, dC};
    const size_t in_sz[5] = {size_t(s->J[0] * s->J[1] * s->J[2]) * e, size_t(s->I[0] * s->I[1] * s->I[2]) * e,
                             size_t(s->J[0] * s->I[0]) * e, size_t(s->J[1] * s->I[1]) * e, size_t(s->J[2] * s->I[2]) * e};
    const size_t out_sz[4] = {in_sz[1], in_sz[2], in_sz[3], in_sz[4]};
    for (int i = 0; i < 5; ++i)
        if (!aligned(ins[i], e)) return TTM_ERR_INVALID_ARG;
    for (int i = 0; i < 4; ++i)
        if (outs[i] && !aligned(outs[i], e)) return TTM_ERR_INVALID_ARG;
    // need only the workspace the requested gradients use; the size query reports the maximum
    BwdPlan p;
    make_bwd_plan(*s, math, dX != nullptr, dA != nullptr, dB != nullptr, dC != nullptr, p);
    if (p.total > 0 && (!ws || ws_bytes < p.total)) return TTM_ERR_WORKSPACE;
    for (int i = 0; i < 4; ++i) {
        if (!outs[i]) continue;
        for (int j = 0; j < 5; ++j)
            if (overlaps(outs[i], out_sz[i], ins[j], in_sz[j])) return TTM_ERR_ALIAS;
        for (int j = i + 1; j < 4; ++j)
            if (outs[j] && overlaps(outs[i], out_sz[i], outs[j], out_sz[j])) return TTM_ERR_ALIAS;
        if (overlaps(outs[i], out_sz[i], ws, p.total)) return TTM_ERR_ALIAS;
    }
    for (int j = 0; j < 5; ++j)
        if (overlaps(ws, p.total, ins[j], in_sz[j])) return TTM_ERR_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(ws);
    if (math == TTM_MATH_F64) return run_backward<M_F64>(p, G, X, A, B, C, dX, dA, dB, dC, w, st);
    return run_backward<M_F32>(p, G, X, A, B, C, dX, dA, dB, dC, w, st);
}

}  // extern "C"
