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
    // float32 with J <= 32, I3 in {256, 512} and I2 a multiple of 4:
    // the three fused kernels (ncg = I3 / 64), with their own workspace layout
    bool fused;
    int ncg;
    size_t f_off_B, f_off_C, f_total;
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

    p.fused = math == TTM_MATH_F32 && p.J1 <= 32 && p.J2 <= 32 && p.J3 <= 32 &&
              (p.I3 == 256 || p.I3 == 512) && p.I2 % 4 == 0 && p.I2 < (int64_t(1) << 24) &&
              p.I1 < (int64_t(1) << 31);
    p.ncg = int(p.I3 / 64);
    off = 0;
    p.f_off_B = take(p.fused, p.I1 * p.J2 * p.I2);
    p.f_off_C = take(p.fused, p.I1 * p.J3 * p.I3);
    p.f_total = off;
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

// ---------------------------------------------------------------------------
// Fused adjoint for float32 with J1, J2, J3 <= 32, I3 in {256, 512} and I2 a
// multiple of 4: two launches in place of the product sequence above.
//
//   k_bwd_xpass_f32    one workgroup per slab X[i1] reads the slab once and
//                      writes dX[i1] once.  With H = G x1 A^T formed in the
//                      workgroup and R = H x2 B^T formed per chunk of rows,
//                      each chunk of X is contracted twice on the matrix cores
//                      (with C for the rows of W = X x3 C, with R for the
//                      slab's share of dC), and dX = R x3 C^T is written for
//                      the same rows.  W never leaves the chip: each chunk of
//                      its rows is contracted with B (the slab's V = X x2 B x3
//                      C) and with H (the slab's columns of its dB share); at
//                      the end dA[:, i1] = G_(1) vec(V).
//   k_bwd_finish_f32   dB and dC as fixed-order sums of the slabs' shares.
//
// The slab streams through LDS in chunks of CR rows x I3 (32 KiB): three
// stages filled by direct-to-LDS copies two chunks ahead, with B's matching
// CR columns in four stages, so that every global read in the loop is a copy
// the kernel waits for explicitly.  Wave (rh, cq) owns row block rh (16 rows)
// and column group cq (64 columns) of each chunk; it reads its 16 x 64 block
// twice: in the W product a lane holds row l % 16 and four consecutive
// columns (the k slots), in the dC product row l / 16 of a k step (the k
// slot) and four consecutive columns (the output columns of four products).
// X words are XOR-swizzled by the row's low four bits so that both reads
// cover all banks.  The W partials of the column groups meet in LDS; their
// V and dB work, and the R of the chunk after next, run in the following
// iteration ahead of its products (double-buffered W partials and R), so one
// barrier per chunk orders everything.  Padded factor rows (j >= J) are
// zeros; rows past I2 read the last row and are masked where they contribute.
// ---------------------------------------------------------------------------
constexpr int FB_THREADS = 512;
constexpr int FB_XSTAGE = 32768;   // bytes of one X chunk

struct FusedArgs {
    const float *X, *A, *B, *C, *G;
    float *partB, *partC;           // workspace: I1 x J2 x I2, I1 x J3 x I3
    float *dX, *dA, *dB, *dC;
    int64_t I1;
    int I2, I3, J1, J2, J3;
    int nbB, nbC;                   // finish kernel: blocks of dB and dC sums
};

template <int NCG>
__global__ void __launch_bounds__(FB_THREADS, 1) k_bwd_xpass_f32(const FusedArgs a) {
    constexpr int NRG = 8 / NCG;                 // 16-row blocks per chunk
    constexpr int CR = 16 * NRG;                 // rows per chunk
    constexpr int I3C = 64 * NCG;
    constexpr int WPR = I3C / 4;                 // 16-byte words per X row
    constexpr int XOPS = FB_XSTAGE / 1024 / 8;   // 16-byte copies per wave per chunk
    constexpr int BSTAGE = 32 * CR * 4;          // bytes of B's chunk: 32 rows j2 x CR columns
    constexpr int BOPS = BSTAGE / 256 / 8;       // 4-byte copies per wave per chunk
    constexpr int WPS = 16 * 33;                 // one wave's W partial tile (padded rows)
    static_assert(NCG == 4 || NCG == 8, "four or eight 64-column groups");
    static_assert(XOPS < 16, "vmcnt range");
    static_assert(32 * FB_THREADS * 4 <= 3 * FB_XSTAGE && 32 * 16 * 4 <= 4 * BSTAGE, "reduction space");

    __shared__ __align__(1024) unsigned char xbuf[3 * FB_XSTAGE];
    __shared__ __align__(256) float bbuf[4][32 * CR];
    __shared__ float rbuf[2][CR * 36];          // R rows padded to 36 floats
    __shared__ float wpart[2][NRG * NCG * WPS];
    __shared__ float hbuf[32 * 33];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rh = wave / NCG, cq = wave % NCG;
    const int h = lane & 15, g = lane >> 4;
    const int64_t i1 = blockIdx.x;
    const int I2 = a.I2, J2 = a.J2, J3 = a.J3;
    const int nch = (I2 + CR - 1) / CR;
    const float *Xs = a.X + i1 * int64_t(I2) * I3C;
    const uint32_t xlds = lds_offset(xbuf), blds = lds_offset(&bbuf[0][0]);

    // chunk c of X into stage c % 3: LDS word q of the stage is row q / WPR,
    // position q % WPR, holding the row's word (q % WPR) ^ (row & 15)
    auto issue_x = [&](int c) __attribute__((always_inline)) {
        const uint32_t st = xlds + uint32_t((c % 3) * FB_XSTAGE);
#pragma unroll
        for (int j = 0; j < XOPS; ++j) {
            const int q = (wave * XOPS + j) * 64 + lane, row = q / WPR, pw = q % WPR;
            const int gr = c * CR + row < I2 ? c * CR + row : I2 - 1;
            dma16_to_lds_m0(Xs + int64_t(gr) * I3C + 4 * (pw ^ (row & 15)), st + uint32_t((wave * XOPS + j) * 1024));
        }
    };
    // B[:, chunk c] into stage c % 4: float p of row j2 holds column
    // c CR + (p ^ bsw(j2)), spreading the 16 rows a fragment read touches
    auto bsw = [](int j2) __attribute__((always_inline)) { return ((j2 * CR) >> 6) & (CR - 1); };
    auto issue_b = [&](int c) __attribute__((always_inline)) {
        const uint32_t st = blds + uint32_t((c & 3) * BSTAGE);
#pragma unroll
        for (int j = 0; j < BOPS; ++j) {
            const int f = (wave * BOPS + j) * 64 + lane, j2 = f / CR, p = f % CR;
            const int col = c * CR + (p ^ bsw(j2));
            const int j2c = j2 < J2 ? j2 : J2 - 1;
            dma4_to_lds_m0(a.B + int64_t(j2c) * I2 + (col < I2 ? col : I2 - 1), st + uint32_t((wave * BOPS + j) * 256));
        }
    };

    // copies of the first chunks, then H[i1] = sum_j1 A[j1][i1] G[j1]
    // (zero-padded to 32 x 32, to LDS and to the workspace for the dX kernel;
    // rows j1 >= J1 read row J1 - 1 with weight zero, so every load is issued
    // before the sums) and the C fragments of the W product
    issue_b(0);
    if (nch > 1) issue_b(1);
    issue_x(0);
    if (nch > 1) issue_x(1);
    {
        const int j3 = tid & 31, j2a = tid >> 5, j2b = j2a + 16;
        const bool va = j2a < J2 && j3 < J3, vb = j2b < J2 && j3 < J3;
        const int64_t gs = int64_t(J2) * J3;
        const float *ga = a.G + (va ? j2a * J3 + j3 : 0), *gb = a.G + (vb ? j2b * J3 + j3 : 0);
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int j1 = 0; j1 < 32; ++j1) {
            const int j1c = j1 < a.J1 ? j1 : a.J1 - 1;
            const float w = j1 < a.J1 ? a.A[int64_t(j1c) * a.I1 + i1] : 0.f;
            s0 += w * ga[j1c * gs];
            s1 += w * gb[j1c * gs];
        }
        s0 = va ? s0 : 0.f;
        s1 = vb ? s1 : 0.f;
        hbuf[j2a * 33 + j3] = s0;
        hbuf[j2b * 33 + j3] = s1;
    }
    // k slot (l/16, e) of step k is column 64 cq + 16 k + 4 (l/16) + e,
    // output column j3 = 16 jb + l % 16
    V16 cf[2][4];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = 16 * jb + h;
            cf[jb][k] = ld16(a.C + int64_t(j < J3 ? j : J3 - 1) * I3C + 64 * cq + 16 * k + 4 * g);
            if (j >= J3) cf[jb][k] = zero16();
        }
    // dX product: k slot (l/16, e) of half hh is j3 = 16 hh + 4 (l/16) + e,
    // column n of product t is i3 = 64 cq + 4 n + t
    V16 cfx[2][4];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 16 * hh + 4 * g + e;
            cfx[hh][e] = ld16(a.C + int64_t(j < J3 ? j : J3 - 1) * I3C + 64 * cq + 4 * h);
            if (j >= J3) cfx[hh][e] = zero16();
        }
    wait_vmcnt<0>();
    __syncthreads();

    // Each wave's share of the work on a chunk's W partials: V piece v =
    // wave (tile v / NRG, row block v % NRG) when v < 4 NRG, and task t:
    // dB tile t (columns 16 (t / NRG).., row block t % NRG) for t < 2 NRG, R
    // tile t - 2 NRG (row block (t - 2 NRG) / 2, columns 16 ((t - 2 NRG) & 1)..)
    // for t < 4 NRG.  Its H operand: hs[k] = H[16 jb2 + l%16][4 k + l/16] for
    // a dB tile, H[4 k + l/16][16 jb3 + l%16] for an R tile.
    const int task = NRG == 1 ? (wave + 4) & 7 : wave;
    const bool has_v = wave < 4 * NRG, is_db = task < 2 * NRG, is_r = !is_db && task < 4 * NRG;
    const int v_t = wave / NRG, v_rb = wave % NRG;
    const int db_jb2 = task / NRG, db_rb = task % NRG;
    const int r_rb = (task - 2 * NRG) >> 1, r_jb3 = (task - 2 * NRG) & 1;
    float hs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        hs[k] = is_db ? hbuf[(16 * db_jb2 + h) * 33 + 4 * k + g]
                      : (is_r ? hbuf[(4 * k + g) * 33 + 16 * r_jb3 + h] : 0.f);

    f32x4 dcacc[2][4], vacc = zero_accv<f32x4>(), dbt = zero_accv<f32x4>(), dxa[4];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int e = 0; e < 4; ++e) dcacc[jb][e] = zero_accv<f32x4>();
    float *pb = a.partB + i1 * int64_t(J2) * I2;

    // R of chunk cn (rows past I2 zero) into rbuf[cn & 1]
    auto r_tiles = [&](int cn) __attribute__((always_inline)) {
        if (!is_r) return;
        const float *bn = bbuf[cn & 3];
        f32x4 acc = zero_accv<f32x4>();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int j2 = 4 * k + g, rho = 16 * r_rb + h;
            acc = mfma_f32(bn[j2 * CR + (rho ^ bsw(j2))], hs[k], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rho = 16 * r_rb + 4 * g + r;
            rbuf[cn & 1][rho * 36 + 16 * r_jb3 + h] = cn * CR + rho < I2 ? acc[r] : 0.f;
        }
    };
    // V and dB of chunk cp from its summed W partials
    auto w_work = [&](int cp) __attribute__((always_inline)) {
        const float *bs = bbuf[cp & 3];
        const float *wp = wpart[cp & 1];
        if (has_v) {
            const int jb2 = v_t >> 1, jb3 = v_t & 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // V[j2][j3] += sum_rows B[j2][row] W[row][j3]
                const int rho = 16 * v_rb + 4 * k + g, j2 = 16 * jb2 + h;
                float av = bs[j2 * CR + (rho ^ bsw(j2))];
                if (cp * CR + rho >= I2) av = 0.f;
                float bv = 0.f;
#pragma unroll
                for (int q = 0; q < NCG; ++q) bv += wp[(v_rb * NCG + q) * WPS + (4 * k + g) * 33 + 16 * jb3 + h];
                vacc = mfma_f32(av, bv, vacc);
            }
        }
        if (is_db) {
            // dB[j2][row] = sum_j3 H[j2][j3] W[row][j3]
            f32x4 acc = zero_accv<f32x4>();
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float bv = 0.f;
#pragma unroll
                for (int q = 0; q < NCG; ++q) bv += wp[(db_rb * NCG + q) * WPS + h * 33 + 4 * k + g];
                acc = mfma_f32(hs[k], bv, acc);
            }
            dbt = acc;
        }
    };
    // stores of results kept in registers: a chunk's dB tile and dX block
    auto store_db = [&](int cp) __attribute__((always_inline)) {
        if (!is_db) return;
        const int col = cp * CR + 16 * db_rb + h;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j2 = 16 * db_jb2 + 4 * g + r;
            if (j2 < J2 && col < I2) pb[int64_t(j2) * I2 + col] = dbt[r];
        }
    };
    float *dXs = a.dX ? a.dX + i1 * int64_t(I2) * I3C + 64 * cq + 4 * h : nullptr;
    auto store_dx = [&](int cp) __attribute__((always_inline)) {
        if (!dXs) return;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = cp * CR + 16 * rh + 4 * g + r;
            const f32x4 v = {dxa[0][r], dxa[1][r], dxa[2][r], dxa[3][r]};
            if (row < I2) __builtin_nontemporal_store(v, reinterpret_cast<f32x4 *>(dXs + int64_t(row) * I3C));
        }
    };

    r_tiles(0);
    for (int c = 0; c < nch; ++c) {
        // X(c) and B(c + 1) have landed when at most the X copies issued in
        // iteration c - 1 (the last copies, after its B copies) are
        // outstanding; stores issued after them only make the wait longer
        if (c + 1 < nch) wait_vmcnt<XOPS>();
        else wait_vmcnt<0>();
        __syncthreads();
        // the previous iterations' results go out ahead of this iteration's
        // copies, so that the next wait finds them older than the copies
        if (c > 0) store_dx(c - 1);
        if (c > 1) store_db(c - 2);
        if (c + 2 < nch) {
            issue_b(c + 2);
            issue_x(c + 2);
        }
        // the previous chunk's W work and the next chunk's R run ahead of
        // this chunk's products (different buffers; the barrier above orders
        // them against both)
        if (c > 0) w_work(c - 1);
        if (c + 1 < nch) r_tiles(c + 1);

        // products on this wave's 16 x 64 block of the chunk
        const float *xs = reinterpret_cast<const float *>(xbuf + (c % 3) * FB_XSTAGE);
        const float *rs = rbuf[c & 1];
        f32x4 wacc[2][2];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) wacc[jb][0] = wacc[jb][1] = zero_accv<f32x4>();
        // dC: k slot = row 16 rh + 4 k + l/16, product e takes column 64 cq + 4 (l%16) + e;
        // W: row 16 rh + l%16, k slot (l/16, e) = column 64 cq + 16 k + 4 (l/16) + e
        const float *xrow_c = xs + (16 * rh + g) * I3C + 64 * cq;
        const float *xrow_w = xs + (16 * rh + h) * I3C + 64 * cq + 4 * (g ^ (h & 3));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            V16 xv, xw;
            xv.u = *reinterpret_cast<const u32x4 *>(xrow_c + 4 * k * I3C + 4 * (h ^ (4 * k + g)));
            xw.u = *reinterpret_cast<const u32x4 *>(xrow_w + 16 * (k ^ (h >> 2)));
            const int rr = 16 * rh + 4 * k + g;
            const float r0 = rs[rr * 36 + h], r1 = rs[rr * 36 + 16 + h];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                dcacc[0][e] = mfma_f32(r0, xv.f[e], dcacc[0][e]);
                dcacc[1][e] = mfma_f32(r1, xv.f[e], dcacc[1][e]);
                wacc[0][k & 1] = mfma_f32(xw.f[e], cf[0][k].f[e], wacc[0][k & 1]);
                wacc[1][k & 1] = mfma_f32(xw.f[e], cf[1][k].f[e], wacc[1][k & 1]);
            }
        }
        float *wp = wpart[c & 1] + (rh * NCG + cq) * WPS;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) wp[(4 * g + r) * 33 + 16 * jb + h] = wacc[jb][0][r] + wacc[jb][1][r];
        // dX[row][i3] = sum_j3 R[row][j3] C[j3][i3] for this wave's block
        if (dXs) {
#pragma unroll
            for (int t = 0; t < 4; ++t) dxa[t] = zero_accv<f32x4>();
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                V16 ra;
                ra.u = *reinterpret_cast<const u32x4 *>(rs + (16 * rh + h) * 36 + 16 * hh + 4 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int t = 0; t < 4; ++t) dxa[t] = mfma_f32(ra.f[e], cfx[hh][e].f[t], dxa[t]);
            }
        }
    }
    store_dx(nch - 1);
    if (nch > 1) store_db(nch - 2);
    __syncthreads();
    w_work(nch - 1);
    store_db(nch - 1);

    // the row blocks' dC shares and the V pieces are added through LDS in a
    // fixed order (no copy is outstanding: the stages are free)
    __syncthreads();
    float *red = reinterpret_cast<float *>(xbuf);
    float *vred = red + (NRG - 1) * NCG * 2048;
    if (rh > 0) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[((rh - 1) * NCG + cq) * 2048 + ((jb * 4 + e) * 4 + r) * 64 + lane] = dcacc[jb][e][r];
    }
    if (has_v)
#pragma unroll
        for (int r = 0; r < 4; ++r) vred[(wave * 4 + r) * 64 + lane] = vacc[r];
    __syncthreads();
    if (rh == 0) {
        for (int q = 1; q < NRG; ++q)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        dcacc[jb][e][r] += red[((q - 1) * NCG + cq) * 2048 + ((jb * 4 + e) * 4 + r) * 64 + lane];
        float *pc = a.partC + i1 * int64_t(J3) * I3C;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j3 = 16 * jb + 4 * g + r;
                if (j3 >= J3) continue;
                const f32x4 v = {dcacc[jb][0][r], dcacc[jb][1][r], dcacc[jb][2][r], dcacc[jb][3][r]};
                *reinterpret_cast<f32x4 *>(pc + int64_t(j3) * I3C + 64 * cq + 4 * h) = v;
            }
    }
    if (!a.dA) return;
    // V[i1] (32 x 32, padded) into hbuf
    if (wave < 4) {
        const int jb2 = wave >> 1, jb3 = wave & 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s = 0.f;
            for (int rb = 0; rb < NRG; ++rb) s += vred[((wave * NRG + rb) * 4 + r) * 64 + lane];
            hbuf[(16 * jb2 + 4 * g + r) * 33 + 16 * jb3 + h] = s;
        }
    }
    __syncthreads();
    // dA[j1][i1] = sum_n G[j1][n] V[i1][n], n = j2 J3 + j3: thread t takes
    // n = t and t + 512 (coalesced rows of G) for every j1; the 512 partial
    // sums of each j1 are then added in thread order, sixteen runs of 32 and
    // then the sixteen run sums
    {
        const int NN = J2 * J3;
        float vv[2];
        int nn[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int n = tid + FB_THREADS * m;
            const bool ok = n < NN;
            nn[m] = ok ? n : 0;
            vv[m] = ok ? hbuf[(n / J3) * 33 + n % J3] : 0.f;
        }
        float *red2 = reinterpret_cast<float *>(xbuf);   // [32 j1][512 threads], after the dC shares were read
        float *red3 = &bbuf[0][0];                      // [32 j1][16 runs]
#pragma unroll
        for (int j1 = 0; j1 < 32; ++j1) {
            const float *gr = a.G + int64_t(j1 < a.J1 ? j1 : a.J1 - 1) * NN;
            red2[j1 * FB_THREADS + tid] = gr[nn[0]] * vv[0] + gr[nn[1]] * vv[1];
        }
        __syncthreads();
        {
            const int j1 = tid >> 4, run = tid & 15;
            float s = 0.f;
            for (int q = 0; q < 32; ++q) s += red2[j1 * FB_THREADS + run * 32 + q];
            red3[j1 * 16 + run] = s;
        }
        __syncthreads();
        if (tid < a.J1) {
            float s = 0.f;
#pragma unroll
            for (int q = 0; q < 16; ++q) s += red3[tid * 16 + q];
            a.dA[int64_t(tid) * a.I1 + i1] = s;
        }
    }
}

// Blocks [0, nbB) and [nbB, nbB + nbC): 64 consecutive elements of dB (or
// dC) each, the sum over i1 of the slabs' shares: 16 groups of consecutive
// i1, each summed in increasing i1 by one thread per 4 elements, then the 16
// group sums in increasing group order.
__global__ void __launch_bounds__(256) k_bwd_finish_f32(const FusedArgs a) {
    __shared__ f32x4 red[16][16];
    const int tid = threadIdx.x, b = blockIdx.x;
    const bool isB = b < a.nbB;
    const int64_t n = isB ? int64_t(a.J2) * a.I2 : int64_t(a.J3) * a.I3;
    const float *part = isB ? a.partB : a.partC;
    float *out = isB ? a.dB : a.dC;
    const int f = tid & 15, grp = tid >> 4;
    const int64_t e4 = (int64_t(isB ? b : b - a.nbB) * 16 + f) * 4;
    const int64_t gs = (a.I1 + 15) / 16, lo = grp * gs, hi = lo + gs < a.I1 ? lo + gs : a.I1;
    f32x4 s = zero_accv<f32x4>();
    if (e4 < n)
        for (int64_t i0 = lo; i0 < hi; i0 += 16) {
            // sixteen loads in flight, added in increasing i1
            f32x4 v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = *reinterpret_cast<const f32x4 *>(part + (i0 + u < hi ? i0 + u : lo) * n + e4);
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (i0 + u < hi) s += v[u];
        }
    red[grp][f] = s;
    __syncthreads();
    if (tid < 16 && e4 < n) {
        f32x4 t = zero_accv<f32x4>();
#pragma unroll
        for (int q = 0; q < 16; ++q) t += red[q][tid];
        *reinterpret_cast<f32x4 *>(out + e4) = t;
    }
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

template <int NCG>
int run_fused_ncg(const FusedArgs &fa, hipStream_t st) {
    int rc = launch("ttm_bwd_xpass", st, [&] {
        hipLaunchKernelGGL(k_bwd_xpass_f32<NCG>, dim3(unsigned(fa.I1)), dim3(FB_THREADS), 0, st, fa);
    });
    if (rc || fa.nbB + fa.nbC == 0) return rc;
    return launch("ttm_bwd_finish", st, [&] {
        hipLaunchKernelGGL(k_bwd_finish_f32, dim3(unsigned(fa.nbB + fa.nbC)), dim3(256), 0, st, fa);
    });
}

int run_fused(const BwdPlan &p, const void *G, const void *X, const void *A, const void *B, const void *C, void *dX,
              void *dA, void *dB, void *dC, unsigned char *ws, hipStream_t st) {
    FusedArgs fa;
    memset(&fa, 0, sizeof fa);
    fa.X = static_cast<const float *>(X);
    fa.A = static_cast<const float *>(A);
    fa.B = static_cast<const float *>(B);
    fa.C = static_cast<const float *>(C);
    fa.G = static_cast<const float *>(G);
    fa.partB = reinterpret_cast<float *>(ws + p.f_off_B);
    fa.partC = reinterpret_cast<float *>(ws + p.f_off_C);
    fa.dX = static_cast<float *>(dX);
    fa.dA = static_cast<float *>(dA);
    fa.dB = static_cast<float *>(dB);
    fa.dC = static_cast<float *>(dC);
    fa.I1 = p.I1;
    fa.I2 = int(p.I2); fa.I3 = int(p.I3);
    fa.J1 = int(p.J1); fa.J2 = int(p.J2); fa.J3 = int(p.J3);
    fa.nbB = dB ? int(ceil_div(p.J2 * p.I2, 64)) : 0;
    fa.nbC = dC ? int(ceil_div(p.J3 * p.I3, 64)) : 0;
    switch (p.ncg) {
        case 4: return run_fused_ncg<4>(fa, st);
        case 8: return run_fused_ncg<8>(fa, st);
        default: return TTM_ERR_UNSUPPORTED;
    }
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
    return std::max(p.total, p.f_total);
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
    // the fused kernels read X, C and write dX 16 bytes at a time
    const bool fused = p.fused && aligned(X, 16) && aligned(C, 16) && (!dX || aligned(dX, 16));
    if (fused) p.total = p.f_total;
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
    if (fused) return run_fused(p, G, X, A, B, C, dX, dA, dB, dC, w, st);
    if (math == TTM_MATH_F64) return run_backward<M_F64>(p, G, X, A, B, C, dX, dA, dB, dC, w, st);
    return run_backward<M_F32>(p, G, X, A, B, C, dX, dA, dB, dC, w, st);
}

}  // extern "C"
