// ttm_hosvd.hip -- the truncated HOSVD factors around the chain, in FP64 on
// the GPU: for each mode n the J_n leading left singular vectors of the
// unfolding X_(n), as the rows of the factor that the chain then applies
// (X x1 U1 x2 U2 x3 U3 is the Tucker core).
//
// Per mode: the Gram matrix G = X_(n) X_(n)^T (I_n x I_n) on the FP64 matrix
// cores (the strided GEMM with a split k range and a fixed-order sum of the
// splits), then its eigendecomposition by the cyclic Jacobi method in one
// workgroup, G resident in LDS (I_n <= 128): each sweep visits every pair
// (p, q) once, in rounds of I_n / 2 disjoint pairs (the round-robin
// schedule), every round one set of plane rotations applied to the rows,
// then the columns, of G.  The rotations are logged (c, s per pair and
// round) instead of being applied to an eigenvector matrix: the product of
// all of them, applied to the unit vectors of the J selected eigenvalues in
// reverse order, gives those J eigenvectors alone, with no pass over an
// n x n matrix in memory per round.
// Sweeps repeat until the off-diagonal mass is below (I_n u)^2 of the
// diagonal's, u = 2^-53 (at most 40): rounding alone keeps it near I_n u^2,
// so a fixed tighter bound would run every sweep.  The eigenvalues sorted in
// decreasing order select the eigenvectors that become the factor's rows,
// each with its entry of largest magnitude made positive (the sign
// convention that makes the vector of a simple eigenvalue unique).
#include <algorithm>
#include <cstring>

#include "ttm_device.hpp"
#include "ttm_gemm.hpp"
#include "ttm_host.hpp"

namespace ttm {

constexpr int EIG_NMAX = 128;
constexpr int EIG_THREADS = 1024;
constexpr int EIG_MAX_SWEEPS = 40;

// The rotation log (per mode: EIG_MAX_SWEEPS * (m - 1) rounds of m / 2
// (c, s) pairs, m = n rounded up to even) and sorted outputs: rows r < J of U
// (J x n) and the n eigenvalues in decreasing order (nullable).  A sits in
// LDS with rows padded to EIG_LDA doubles, so that the column updates of a
// round (32 consecutive rows of one column per half-wave) hit distinct banks.
// Thread t of a rotation phase takes pair t / 16 and elements (t % 16) + 16 m.
constexpr int EIG_LDA = EIG_NMAX + 1;
constexpr int EIG_RB = 8;    // rounds of rotations per prefetched block when rebuilding the eigenvectors
// One workgroup per mode (the three solves are independent).
struct JacobiArgs {
    const double *G[3];
    double2 *log[3];
    double *U[3], *evals[3];
    int n[3], J[3];
};

// Players p, q of pair k in round r of the round-robin schedule over m
// players (m even): player m - 1 stays, the others rotate.
__device__ __forceinline__ void rr_pair(int r, int k, int m, int &p, int &q) {
    if (k == 0) { p = r; q = m - 1; }
    else { p = (r + k) % (m - 1); q = (r - k + (m - 1)) % (m - 1); }
}
__global__ void __launch_bounds__(EIG_THREADS) k_sym_jacobi(const JacobiArgs ja) {
    const int mode = blockIdx.x;
    const double *G = ja.G[mode];
    double2 *rlog = ja.log[mode];
    double *U = ja.U[mode], *evals = ja.evals[mode];
    const int n = ja.n[mode], J = ja.J[mode];
    __shared__ double A[EIG_NMAX * EIG_LDA];
    __shared__ double rc[EIG_NMAX / 2 + 1], rs[EIG_NMAX / 2 + 1];
    __shared__ int rp[EIG_NMAX / 2 + 1], rq[EIG_NMAX / 2 + 1];
    __shared__ double red[EIG_THREADS / 64][2];
    __shared__ int order[EIG_NMAX];
    __shared__ int done;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < n * n; e += EIG_THREADS) {
        const int i = e / n, j = e - i * n;
        A[i * EIG_LDA + j] = G[e];
    }
    const int m = n + (n & 1);          // players of the round-robin (one idle slot when n is odd)
    const int np = m / 2;
    const int pk = tid >> 4, e0 = tid & 15;   // pair and first element of this thread
    int rounds = 0;                     // rounds logged
    __syncthreads();
    for (int sweep = 0; sweep < EIG_MAX_SWEEPS; ++sweep) {
        for (int r = 0; r < m - 1; ++r, ++rounds) {
            // rotation of every pair of this round
            if (tid < np) {
                int p, q;
                rr_pair(r, tid, m, p, q);
                double c = 1.0, s = 0.0;
                if (p < n && q < n) {
                    const double apq = A[p * EIG_LDA + q];
                    if (apq != 0.0) {
                        const double tau = (A[q * EIG_LDA + q] - A[p * EIG_LDA + p]) / (2.0 * apq);
                        const double at = fabs(tau);
                        const double t = at > 1e150 ? 0.5 / tau
                                                    : (tau >= 0.0 ? 1.0 : -1.0) / (at + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                rp[tid] = p;
                rq[tid] = q;
                rc[tid] = c;
                rs[tid] = s;
                rlog[int64_t(rounds) * np + tid] = double2{c, s};
            }
            __syncthreads();
            const int p = pk < np ? rp[pk] : n, q = pk < np ? rq[pk] : n;
            const bool live = p < n && q < n;
            const double c = live ? rc[pk] : 1.0, s = live ? rs[pk] : 0.0;
            constexpr int EPT = EIG_NMAX / 16;   // elements per thread
            // rows p and q of A
            if (live)
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const int j = e0 + 16 * u;
                    if (j < n) {
                        const double ap = A[p * EIG_LDA + j], aq = A[q * EIG_LDA + j];
                        A[p * EIG_LDA + j] = c * ap - s * aq;
                        A[q * EIG_LDA + j] = s * ap + c * aq;
                    }
                }
            __syncthreads();
            // columns p and q of A
            if (live)
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const int i = e0 + 16 * u;
                    if (i < n) {
                        const double ap = A[i * EIG_LDA + p], aq = A[i * EIG_LDA + q];
                        A[i * EIG_LDA + p] = c * ap - s * aq;
                        A[i * EIG_LDA + q] = s * ap + c * aq;
                    }
                }
            __syncthreads();
        }
        // off-diagonal and diagonal mass, fixed-order reduction
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            const double v = A[i * EIG_LDA + j];
            if (i == j) dia += v * v;
            else off += v * v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            dia += __shfl_xor(dia, o);
        }
        if (lane == 0) { red[wave][0] = off; red[wave][1] = dia; }
        __syncthreads();
        if (tid == 0) {
            double so = 0.0, sd = 0.0;
            for (int w = 0; w < EIG_THREADS / 64; ++w) { so += red[w][0]; sd += red[w][1]; }
            // rounding keeps the off-diagonal mass near n u^2 of the
            // diagonal's (u = 2^-53): stop at (n u)^2, a hundred times above
            const double nu = double(n) * 0x1p-53;
            done = so <= nu * nu * sd;
        }
        __syncthreads();
        if (done) break;
    }
    // decreasing order of the eigenvalues (ties: lower index first)
    if (tid < n) {
        const double li = A[tid * EIG_LDA + tid];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j * EIG_LDA + j];
            rank += (lj > li || (lj == li && j < tid)) ? 1 : 0;
        }
        order[rank] = tid;
    }
    __syncthreads();
    if (evals && tid < n) evals[tid] = A[order[tid] * EIG_LDA + order[tid]];
    // Eigenvector of eigenvalue order[j], j < J: the rounds' rotations Q_k
    // (rows p, q of a vector: x_p <- c x_p - s x_q, x_q <- s x_p + c x_q)
    // turned the identity into the matrix whose rows are the eigenvectors,
    // Q_K ... Q_1, so row order[j] is e^T Q_K ... Q_1 with e = e_order[j]:
    // Q_K^T first, down to Q_1^T, on a vector started at e.  The vectors
    // take A's place (its diagonal is read above); thread t owns pair t % 64
    // of every round for the vectors t / 64, t / 64 + 16, ...  Each thread
    // holds the (c, s) of its pair for a block of EIG_RB rounds and loads the
    // next block while it applies the current one.
    __syncthreads();
    double *x = A;                      // J vectors of n, stride EIG_LDA
    for (int e = tid; e < J * n; e += EIG_THREADS) {
        const int j = e / n, i = e - j * n;
        x[j * EIG_LDA + i] = i == order[j] ? 1.0 : 0.0;
    }
    const int k = tid & 63, j0 = tid >> 6;
    const bool kin = k < np;
    double2 cur[EIG_RB], nxt[EIG_RB];
    auto load_block = [&](int top, double2 (&dst)[EIG_RB]) {   // rounds top, top - 1, ..., top - EIG_RB + 1
#pragma unroll
        for (int b = 0; b < EIG_RB; ++b) {
            const int rd = top - b;
            dst[b] = (kin && rd >= 0) ? rlog[int64_t(rd) * np + k] : double2{1.0, 0.0};
        }
    };
    load_block(rounds - 1, cur);
    __syncthreads();
    for (int top = rounds - 1; top >= 0; top -= EIG_RB) {
        if (top - EIG_RB >= 0) load_block(top - EIG_RB, nxt);
#pragma unroll
        for (int b = 0; b < EIG_RB; ++b) {
            const int rd = top - b;
            if (rd >= 0) {
                int p, q;
                rr_pair(rd % (m - 1), k, m, p, q);
                if (kin && p < n && q < n) {
                    const double c = cur[b].x, s = cur[b].y;
                    for (int j = j0; j < J; j += EIG_THREADS / 64) {
                        const double xp = x[j * EIG_LDA + p], xq = x[j * EIG_LDA + q];
                        x[j * EIG_LDA + p] = c * xp + s * xq;
                        x[j * EIG_LDA + q] = c * xq - s * xp;
                    }
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int b = 0; b < EIG_RB; ++b) cur[b] = nxt[b];
    }
    // factor rows: one wave per row, sign fixed by the entry of largest magnitude
    for (int row = wave; row < J; row += EIG_THREADS / 64) {
        const double *v = x + row * EIG_LDA;
        double best = -1.0;
        int bi = n;
        for (int i = lane; i < n; i += 64) {
            const double a = fabs(v[i]);
            if (a > best || (a == best && i < bi)) { best = a; bi = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o);
            const int oi = __shfl_xor(bi, o);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const double sgn = v[bi] < 0.0 ? -1.0 : 1.0;
        for (int i = lane; i < n; i += 64) U[int64_t(row) * n + i] = sgn * v[i];
    }
}

struct HosvdPlan {
    int64_t nmax;
    int ks[3];
    size_t off_G[3], off_L[3], off_P, total;
};

static void hosvd_plan(const ttm_shape &s, HosvdPlan &p) {
    p.nmax = std::max(s.I[0], std::max(s.I[1], s.I[2]));
    const int64_t KT = GemmCfg<M_F64>::KT;
    int kmax = 1;
    for (int n = 0; n < 3; ++n) {
        const int64_t K = s.I[0] * s.I[1] * s.I[2] / s.I[n];
        const int64_t tiles = ceil_div(s.I[n], 64) * ceil_div(s.I[n], 64);
        // about 256 workgroups in all, each split at least eight chunks long
        int64_t k = std::min<int64_t>(ceil_div(256, tiles), ceil_div(K, 8 * KT));
        k = std::max<int64_t>(1, std::min<int64_t>(k, 64));
        p.ks[n] = int(k);
        kmax = std::max(kmax, p.ks[n]);
    }
    const size_t nn = size_t(p.nmax * p.nmax) * 8, nn_al = (nn + 255) & ~size_t(255);
    // rotation log: every round of the largest mode, (c, s) per pair
    const int64_t mmax = p.nmax + (p.nmax & 1);
    const size_t lg = size_t(EIG_MAX_SWEEPS) * size_t(std::max<int64_t>(mmax - 1, 1)) * size_t(mmax / 2) * 16;
    const size_t lg_al = (lg + 255) & ~size_t(255);
    for (int n = 0; n < 3; ++n) {
        p.off_G[n] = size_t(n) * nn_al;
        p.off_L[n] = 3 * nn_al + size_t(n) * lg_al;
    }
    p.off_P = 3 * nn_al + 3 * lg_al;
    p.total = p.off_P + (kmax > 1 ? size_t(kmax) * nn : 0);
}

static int gram_f64(const ttm_shape &s, const double *X, int mode, double *G, double *part, int ks, hipStream_t st) {
    const int64_t I1 = s.I[0], I2 = s.I[1], I3 = s.I[2];
    const int64_t n = s.I[mode - 1];
    GemmArgs a;
    memset(&a, 0, sizeof a);
    a.A = X;
    a.B = X;
    a.P = 1;
    a.M = n;
    a.N = n;
    if (mode == 1) {
        a.K = I2 * I3; a.Ki = a.K;
        a.sam = I2 * I3; a.saki = 1;
        a.sbn = I2 * I3; a.sbki = 1;
    } else if (mode == 2) {
        a.K = I1 * I3; a.Ki = I3;
        a.sam = I3; a.sako = I2 * I3; a.saki = 1;
        a.sbn = I3; a.sbko = I2 * I3; a.sbki = 1;
    } else {
        a.K = I1 * I2; a.Ki = a.K;
        a.sam = 1; a.saki = I3;
        a.sbn = 1; a.sbki = I3;
    }
    const int64_t KT = GemmCfg<M_F64>::KT;
    a.k_per_split = round_up(ceil_div(a.K, ks), KT);
    const int nsplit = int(ceil_div(a.K, a.k_per_split));
    a.C = nsplit > 1 ? static_cast<void *>(part) : static_cast<void *>(G);
    a.scm = n;
    a.scn = 1;
    a.scs = n * n;
    dim3 grid(unsigned(ceil_div(n, 64) * ceil_div(n, 64)), unsigned(nsplit), 1);
    int rc = launch("ttm_gram", st, [&] { hipLaunchKernelGGL((k_gemm<M_F64, false, false>), grid, dim3(256), 0, st, a); });
    if (rc || nsplit == 1) return rc;
    return launch("ttm_gram_sum", st, [&] {
        hipLaunchKernelGGL(k_sum_splits<double>, dim3(unsigned(ceil_div(n * n, 256))), dim3(256), 0, st, part, n * n,
                           nsplit, n * n, G);
    });
}

static int hosvd_check_shape(const ttm_shape *s) {
    if (!s) return TTM_ERR_INVALID_ARG;
    for (int n = 0; n < 3; ++n) {
        if (s->I[n] < 1 || s->J[n] < 1 || s->J[n] > s->I[n]) return TTM_ERR_INVALID_ARG;
        if (s->I[n] > EIG_NMAX) return TTM_ERR_UNSUPPORTED;
    }
    return TTM_OK;
}

}  // namespace ttm

using namespace ttm;

extern "C" {

size_t ttm_hosvd_workspace_size(const ttm_shape *shape) {
    if (hosvd_check_shape(shape) != TTM_OK) return 0;
    HosvdPlan p;
    hosvd_plan(*shape, p);
    return p.total;
}

int ttm_hosvd(const ttm_shape *shape, const void *X, void *A, void *B, void *C, void *evals, void *ws,
              size_t ws_bytes, void *stream) {
    int rc = hosvd_check_shape(shape);
    if (rc) return rc;
    if (!X || !A || !B || !C) return TTM_ERR_INVALID_ARG;
    if (!aligned(X, 8) || !aligned(A, 8) || !aligned(B, 8) || !aligned(C, 8) || (evals && !aligned(evals, 8)))
        return TTM_ERR_INVALID_ARG;
    HosvdPlan p;
    hosvd_plan(*shape, p);
    if (!ws || ws_bytes < p.total) return TTM_ERR_WORKSPACE;
    if (!aligned(ws, 16)) return TTM_ERR_INVALID_ARG;
    const ttm_shape &s = *shape;
    const size_t nx = size_t(s.I[0] * s.I[1] * s.I[2]) * 8;
    void *outs[3] = {A, B, C};
    for (int n = 0; n < 3; ++n) {
        const size_t nu = size_t(s.J[n] * s.I[n]) * 8;
        if (overlaps(outs[n], nu, X, nx) || overlaps(outs[n], nu, ws, p.total)) return TTM_ERR_ALIAS;
        for (int k = 0; k < n; ++k)
            if (overlaps(outs[n], nu, outs[k], size_t(s.J[k] * s.I[k]) * 8)) return TTM_ERR_ALIAS;
    }
    if (overlaps(ws, p.total, X, nx)) return TTM_ERR_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(ws);
    double *part = reinterpret_cast<double *>(w + p.off_P);
    JacobiArgs ja;
    int64_t eoff = 0;
    for (int n = 0; n < 3; ++n) {
        double *G = reinterpret_cast<double *>(w + p.off_G[n]);
        if ((rc = gram_f64(s, static_cast<const double *>(X), n + 1, G, part, p.ks[n], st))) return rc;
        ja.G[n] = G;
        ja.log[n] = reinterpret_cast<double2 *>(w + p.off_L[n]);
        ja.U[n] = static_cast<double *>(outs[n]);
        ja.evals[n] = evals ? static_cast<double *>(evals) + eoff : nullptr;
        ja.n[n] = int(s.I[n]);
        ja.J[n] = int(s.J[n]);
        eoff += s.I[n];
    }
    // the three eigensolves side by side, one workgroup each
    return launch("ttm_sym_jacobi", st, [&] {
        hipLaunchKernelGGL(k_sym_jacobi, dim3(3), dim3(EIG_THREADS), 0, st, ja);
    });
}

}  // extern "C"
