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
};

constexpr int64_t KT_F32 = 32, KT_F64 = 16;

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
    if (dA) {
        SplitK k = choose_split(p.J1, p.I1, p.NN, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, int64_t(k.ks) * p.J1 * p.I1);
    }
    if (dB) {
        SplitK k = choose_split(p.J2, p.I2, p.I1 * p.J3, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, int64_t(k.ks) * p.J2 * p.I2);
    }
    if (dC) {
        SplitK k = choose_split(p.J3, p.I3, p.I1 * p.I2, 1, KT);
        if (k.ks > 1) p.part_elems = std::max(p.part_elems, int64_t(k.ks) * p.J3 * p.I3);
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
    int rc = TTM_OK;
    if (p.need_w) {   // W[(i1,i2)][j3] = sum_i3 X[(i1,i2)][i3] C[j3][i3]
        GemmArgs a = gargs();
        a.A = X; a.B = C; a.C = W;
        a.M = I1 * I2; a.N = J3; a.K = I3;
        a.sam = I3; a.saki = 1;
        a.sbn = I3; a.sbki = 1;
        a.scm = J3; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, 1, false, nullptr, st, "ttm_bwd_W"))) return rc;
    }
    if (p.need_v) {   // V[i1][j2][j3] = sum_i2 B[j2][i2] W[i1][i2][j3]
        GemmArgs a = gargs();
        a.A = B; a.B = W; a.C = V;
        a.M = J2; a.N = J3; a.K = I2;
        a.sam = I2; a.saki = 1;
        a.sbb = I2 * J3; a.sbki = J3; a.sbn = 1;
        a.scb = NN; a.scm = J3; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, I1, false, nullptr, st, "ttm_bwd_V"))) return rc;
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
        if ((rc = run_gemm<MATH>(a, I1, false, nullptr, st, "ttm_bwd_R"))) return rc;
    }
    if (dX) {         // dX[(i1,i2)][i3] = sum_j3 R[(i1,i2)][j3] C[j3][i3]
        GemmArgs a = gargs();
        a.A = R; a.B = C; a.C = dX;
        a.M = I1 * I2; a.N = I3; a.K = J3;
        a.sam = J3; a.saki = 1;
        a.sbn = 1; a.sbki = I3;
        a.scm = I3; a.scn = 1;
        if ((rc = run_gemm<MATH>(a, 1, false, nullptr, st, "ttm_bwd_dX"))) return rc;
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
        if ((rc = run_gemm<MATH>(a, 1, true, Pt, st, "ttm_bwd_dC"))) return rc;
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
