// ttm_compact.hip -- the compact sixth-order first derivative of Sec. 4.2,
// Eq. (cfds), applied along one mode of a periodic 3-way field without forming
// D = A_c^-1 B_c.  Two solvers of the cyclic tridiagonal system:
//
// Single pass (fibers of at least 2K points and a multiple of 8, K = 40 in
// float64, 24 in float32, and |alpha| small enough that rho^K is below the
// rounding unit): the circulant factorization of A_c below turns the solve
// into two first-order recursions that forget their start after K points, so
// each point is read once and written once (the algorithmic two transfers).
//
// Exact sweeps (shorter fibers): the five-point right-hand side is built on
// the fly and fused with the forward pass of a cyclic tridiagonal solve
// (Sec. 2.1, the periodic Thomas algorithm, here as a Sherman-Morrison
// correction of one tridiagonal solve); the correction's scalar is
// accumulated during the forward pass, so one backward pass finishes the
// solve.  Splitting (gamma = -1): A_c = T + p q^T, T tridiagonal with alpha
// beside the diagonal and diagonal 1 except T_00 = 1 - gamma, T_{n-1,n-1} =
// 1 - alpha^2 / gamma; p = (gamma, 0, .., 0, alpha), q = (1, 0, .., 0, alpha /
// gamma).  With T y = d and T z = p the solution is x = y - [q.y / (1 + q.z)]
// z.  The fiber-independent data -- inv_j and cp_j of T's forward pass, z, and
// weights w_j with y_0 = sum_j w_j y'_j (y' the forward-pass values) -- come
// from one device thread in double precision before the sweep.  The forward
// pass stores y' into Y and the backward pass turns it into the solution in
// place: four transfers per point.
//
// Layout: one lane per fiber for modes 1 and 2, as the paper gives each GPU
// thread one line of a group of SZ lines (Sec. 4.1): row-major X makes those
// fibers interleaved already (lane f and f+1 read neighbouring addresses at
// every step).  Mode-3 fibers are contiguous rows, moved through LDS tiles.
#include <math.h>

#include <algorithm>

#include "ttm_device.hpp"
#include "ttm_host.hpp"

namespace ttm {

namespace {

constexpr int64_t COMPACT_PREP_LDS_MAX = 8192;   // fibers up to this length keep the prep in LDS

struct CompactArgs {
    int64_t n, stride, nfib, i3;   // fiber length and element stride; fibers; I3 (mode 2 mapping)
    int64_t s12;                   // I2 * I3
    int mode;
    double ca, cb, alpha;          // a / (2h), b / (4h), alpha
};

// ws layout (elements of T): inv[n] | cp[n] | w[n] | z[n] | k, alpha/gamma.
// One thread runs the forward pass of T (and of T z = p) in double, keeping
// z' and cp in LDS when they fit (dynamic LDS of 16 n bytes, else read back
// from the workspace), then z's backward pass.
template <typename T>
__global__ void __launch_bounds__(64) k_compact_prep(int64_t n, double alpha, T *ws) {
    extern __shared__ __align__(16) unsigned char smem_prep[];
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double gamma = -1.0;
    T *inv = ws, *cp = ws + n, *w = ws + 2 * n, *z = ws + 3 * n;
    const bool lds = n <= COMPACT_PREP_LDS_MAX;
    double *zl = reinterpret_cast<double *>(smem_prep), *cl = zl + (lds ? n : 0);
    double cprev = 0.0, zf = 0.0, wj = 1.0;
    for (int64_t j = 0; j < n; ++j) {
        const double dj = (j == 0) ? 1.0 - gamma : (j == n - 1 ? 1.0 - alpha * alpha / gamma : 1.0);
        const double iv = 1.0 / (dj - (j > 0 ? alpha * cprev : 0.0));
        const double pj = (j == 0) ? gamma : (j == n - 1 ? alpha : 0.0);
        zf = (pj - (j > 0 ? alpha * zf : 0.0)) * iv;
        if (j > 0) wj = -cprev * wj;
        cprev = alpha * iv;
        inv[j] = T(iv);
        cp[j] = T(cprev);
        w[j] = T(wj);
        if (lds) { zl[j] = zf; cl[j] = cprev; }
        else z[j] = T(zf);                // forward value, replaced below
    }
    const double zlast = zf;              // z_{n-1} = z'_{n-1}
    double zn = zlast;
    z[n - 1] = T(zn);
    for (int64_t j = n - 2; j >= 0; --j) {
        zn = (lds ? zl[j] - cl[j] * zn : double(z[j]) - double(cp[j]) * zn);
        z[j] = T(zn);
    }
    ws[4 * n] = T(1.0 / (1.0 + zn + (alpha / gamma) * zlast));   // zn = z_0 here
    ws[4 * n + 1] = T(alpha / gamma);
}

template <typename T>
__global__ void __launch_bounds__(256) k_compact(const CompactArgs a, const T *__restrict__ X, T *__restrict__ Y,
                                                 const T *__restrict__ ws) {
    for (int64_t f = int64_t(blockIdx.x) * 256 + threadIdx.x; f < a.nfib; f += int64_t(gridDim.x) * 256) {
    int64_t base;
    if (a.mode == 1) base = f;
    else if (a.mode == 2) base = (f / a.i3) * a.s12 + f % a.i3;
    else base = f * a.n;
    const int64_t n = a.n, s = a.stride;
    const T *u = X + base;
    T *y = Y + base;
    const T *inv = ws, *cp = ws + n, *w = ws + 2 * n, *z = ws + 3 * n;
    const T kk = ws[4 * n], ag = ws[4 * n + 1];
    const T ca = T(a.ca), cb = T(a.cb), alpha = T(a.alpha);

    // forward: d_j from the window u_{j-2} .. u_{j+2} (indices mod n), then
    // y'_j = (d_j - alpha y'_{j-1}) inv_j, stored in Y; q.y accumulates
    const T u0 = u[0], u1 = u[s];
    T um2 = u[(n - 2) * s], um1 = u[(n - 1) * s], uc = u0, up1 = u1;
    T yp = T(0), acc = T(0);
#pragma unroll 4
    for (int64_t j = 0; j < n; ++j) {
        const int64_t j2 = j + 2;
        const T up2 = j2 < n ? u[j2 * s] : (j2 == n ? u0 : u1);
        const T d = ca * (up1 - um1) + cb * (up2 - um2);
        yp = (d - alpha * yp) * inv[j];
        y[j * s] = yp;
        acc += w[j] * yp;
        um2 = um1;
        um1 = uc;
        uc = up1;
        up1 = up2;
    }
    // Sherman-Morrison scalar: q.y / (1 + q.z) with y_0 = acc, y_{n-1} = y'_{n-1}
    const T sc = kk * (acc + ag * yp);
    // backward: y_j = y'_j - cp_j y_{j+1}; x_j = y_j - sc z_j
    T yn = yp;
    y[(n - 1) * s] = yn - sc * z[n - 1];
#pragma unroll 4
    for (int64_t j = n - 2; j >= 0; --j) {
        yn = y[j * s] - cp[j] * yn;
        y[j * s] = yn - sc * z[j];
    }
    }
}

// Mode 3: the fibers are contiguous rows.  A wave owns 64 rows; tiles of
// 64 rows x RT points (128 bytes per row) go through LDS so that every global
// access is a coalesced 16-byte-per-lane load or store, while each lane still
// walks its own row.  Forward tiles carry a two-point halo (taken modulo n).
// Per-wave LDS: an input tile and an output tile, rows padded by one element.
template <typename T>
struct RowsCfg {
    static constexpr int VE = 16 / int(sizeof(T));    // elements per 16-byte word
    static constexpr int RT = 128 / int(sizeof(T));   // points per tile row
    static constexpr int WPR = RT / VE;               // 16-byte words per tile row
    static constexpr int LD = RT + 3;                 // LDS row stride (tile + halo + pad)
    static constexpr int WAVE_ELEMS = 2 * 64 * LD;
};

template <typename T>
__global__ void __launch_bounds__(256) k_compact_rows(const CompactArgs a, const T *__restrict__ X,
                                                      T *__restrict__ Y, const T *__restrict__ ws) {
    typedef RowsCfg<T> CF;
    constexpr int VE = CF::VE, RT = CF::RT, LD = CF::LD;
    extern __shared__ __align__(16) unsigned char smem_rows[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    T *tin = reinterpret_cast<T *>(smem_rows) + wave * CF::WAVE_ELEMS;
    T *tout = tin + 64 * LD;
    const int64_t n = a.n;
    const int64_t row0 = (int64_t(blockIdx.x) * (blockDim.x >> 6) + wave) * 64;
    if (row0 >= a.nfib) return;                       // whole wave: no LDS shared across waves
    const int64_t nrows = a.nfib - row0 < 64 ? a.nfib - row0 : 64;
    const T *inv = ws, *cp = ws + n, *w = ws + 2 * n, *z = ws + 3 * n;
    const T kk = ws[4 * n], ag = ws[4 * n + 1];
    const T ca = T(a.ca), cb = T(a.cb), alpha = T(a.alpha);
    const int64_t myrow = row0 + (lane < nrows ? lane : nrows - 1);
    const T *urow = X + myrow * n;

    // cooperative tile transfer: lane l moves word l % WPR of rows l / WPR + (64 / WPR) i
    constexpr int WPR = CF::WPR, RPP = 64 / WPR;
    const int wl = lane % WPR, rl = lane / WPR;
    auto load_tile = [&](const T *src, int64_t t0, int cols) {
#pragma unroll
        for (int i = 0; i < WPR; ++i) {
            const int r = rl + RPP * i;
            const int c = wl * VE;
            if (r < nrows && c < cols) {
                const T *g = src + (row0 + r) * n + t0 + c;
                if (c + VE <= cols) {
                    V16 v = ld16(g);
#pragma unroll
                    for (int e = 0; e < VE; ++e) tin[r * LD + c + e] = reinterpret_cast<const T *>(&v)[e];
                } else {
                    for (int e = 0; c + e < cols; ++e) tin[r * LD + c + e] = g[e];
                }
            }
        }
    };
    auto store_tile = [&](T *dst, int64_t t0, int cols) {
#pragma unroll
        for (int i = 0; i < WPR; ++i) {
            const int r = rl + RPP * i;
            const int c = wl * VE;
            if (r < nrows && c < cols) {
                T *g = dst + (row0 + r) * n + t0 + c;
                if (c + VE <= cols) {
                    V16 v;
#pragma unroll
                    for (int e = 0; e < VE; ++e) reinterpret_cast<T *>(&v)[e] = tout[r * LD + c + e];
                    *reinterpret_cast<u32x4 *>(g) = v.u;
                } else {
                    for (int e = 0; c + e < cols; ++e) g[e] = tout[r * LD + c + e];
                }
            }
        }
    };

    // forward sweep over tiles [t0, t0 + cols), halo points t0 + cols, t0 + cols + 1 (mod n)
    T um2 = urow[n - 2], um1 = urow[n - 1], uc = urow[0], up1 = urow[1];
    T yp = T(0), acc = T(0);
    for (int64_t t0 = 0; t0 < n; t0 += RT) {
        const int cols = int(n - t0 < RT ? n - t0 : RT);
        wave_sync();
        load_tile(X, t0, cols);
        // the two halo points of each row (scalar loads, modulo n)
        for (int e = lane; e < 2 * nrows; e += 64) {
            const int r = e >> 1, h = e & 1;
            int64_t c = t0 + cols + h;
            if (c >= n) c -= n;
            tin[r * LD + cols + h] = X[(row0 + r) * n + c];
        }
        wave_sync();
        const T *mine = tin + lane * LD;
        for (int c = 0; c < cols; ++c) {
            const int64_t j = t0 + c;
            const T up2 = mine[c + 2];
            const T d = ca * (up1 - um1) + cb * (up2 - um2);
            yp = (d - alpha * yp) * inv[j];
            tout[lane * LD + c] = yp;
            acc += w[j] * yp;
            um2 = um1;
            um1 = uc;
            uc = up1;
            up1 = up2;
        }
        wave_sync();
        store_tile(Y, t0, cols);
    }
    const T sc = kk * (acc + ag * yp);

    // backward sweep over the same tiles in reverse, in place in Y
    T yn = T(0);
    const int64_t last0 = ((n - 1) / RT) * RT;
    for (int64_t t0 = last0; t0 >= 0; t0 -= RT) {
        const int cols = int(n - t0 < RT ? n - t0 : RT);
        wave_sync();
        load_tile(Y, t0, cols);
        wave_sync();
        const T *mine = tin + lane * LD;
        for (int c = cols - 1; c >= 0; --c) {
            const int64_t j = t0 + c;
            yn = mine[c] - (j == n - 1 ? T(0) : cp[j]) * yn;
            tout[lane * LD + c] = yn - sc * z[j];
        }
        wave_sync();
        store_tile(Y, t0, cols);
    }
}

// The same sweeps for n a multiple of RT (every tile whole): the next tile
// and its halo are loaded into registers while the current one is computed,
// and the RT steps of a tile are unrolled with the tile's coefficients read
// before the recurrence starts.
template <typename T>
__global__ void __launch_bounds__(256) k_compact_rows_full(const CompactArgs a, const T *__restrict__ X,
                                                           T *__restrict__ Y, const T *__restrict__ ws) {
    typedef RowsCfg<T> CF;
    constexpr int VE = CF::VE, RT = CF::RT, LD = CF::LD, WPR = CF::WPR, RPP = 64 / WPR;
    extern __shared__ __align__(16) unsigned char smem_rows[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    T *tin = reinterpret_cast<T *>(smem_rows) + wave * CF::WAVE_ELEMS;
    T *tout = tin + 64 * LD;
    const int64_t n = a.n, ntiles = n / RT;
    const int64_t row0 = (int64_t(blockIdx.x) * (blockDim.x >> 6) + wave) * 64;
    if (row0 >= a.nfib) return;                       // whole wave: no LDS shared across waves
    const int nrows = int(a.nfib - row0 < 64 ? a.nfib - row0 : 64);
    const T *inv = ws, *cp = ws + n, *w = ws + 2 * n, *z = ws + 3 * n;
    const T kk = ws[4 * n], ag = ws[4 * n + 1];
    const T ca = T(a.ca), cb = T(a.cb), alpha = T(a.alpha);
    const int64_t myrow = row0 + (lane < nrows ? lane : nrows - 1);
    const T *urow = X + myrow * n;

    // lane l moves word l % WPR of rows l / WPR + RPP i (rows past the range
    // re-read the last row and are not stored); halo values: lane l holds
    // point t0 + RT + (l & 1) (mod n) of row l / 2 and of row 32 + l / 2
    const int wl = lane % WPR, rl = lane / WPR;
    V16 buf[WPR];
    T halo[2];
    auto rowc = [&](int r) -> int64_t { return row0 + (r < nrows ? r : nrows - 1); };
    auto fetch = [&](const T *src, int64_t t0, bool with_halo) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < WPR; ++i) buf[i] = ld16(src + rowc(rl + RPP * i) * n + t0 + wl * VE);
        if (with_halo) {
            int64_t c = t0 + RT + (lane & 1);
            if (c >= n) c -= n;
#pragma unroll
            for (int h = 0; h < 2; ++h) halo[h] = src[rowc(32 * h + (lane >> 1)) * n + c];
        }
    };
    auto put = [&](bool with_halo) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < WPR; ++i) {
            const int r = rl + RPP * i;
#pragma unroll
            for (int e = 0; e < VE; ++e) tin[r * LD + wl * VE + e] = reinterpret_cast<const T *>(&buf[i])[e];
        }
        if (with_halo) {
#pragma unroll
            for (int h = 0; h < 2; ++h) tin[(32 * h + (lane >> 1)) * LD + RT + (lane & 1)] = halo[h];
        }
    };
    auto store_tile = [&](int64_t t0) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < WPR; ++i) {
            const int r = rl + RPP * i;
            if (r < nrows) {
                V16 v;
#pragma unroll
                for (int e = 0; e < VE; ++e) reinterpret_cast<T *>(&v)[e] = tout[r * LD + wl * VE + e];
                *reinterpret_cast<u32x4 *>(Y + (row0 + r) * n + t0 + wl * VE) = v.u;
            }
        }
    };

    // forward sweep
    T um2 = urow[n - 2], um1 = urow[n - 1], uc = urow[0], up1 = urow[1];
    T yp = T(0), acc = T(0);
    fetch(X, 0, true);
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t t0 = t * RT;
        wave_sync();
        put(true);
        wave_sync();
        T u[RT + 2];
        const T *mine = tin + lane * LD;
#pragma unroll
        for (int c = 0; c < RT + 2; ++c) u[c] = mine[c];
        if (t + 1 < ntiles) fetch(X, t0 + RT, true);
        T ci[RT], cw[RT];
#pragma unroll
        for (int c = 0; c < RT; ++c) {
            ci[c] = inv[t0 + c];
            cw[c] = w[t0 + c];
        }
#pragma unroll
        for (int c = 0; c < RT; ++c) {
            const T up2 = u[c + 2];
            const T d = ca * (up1 - um1) + cb * (up2 - um2);
            yp = (d - alpha * yp) * ci[c];
            tout[lane * LD + c] = yp;
            acc += cw[c] * yp;
            um2 = um1;
            um1 = uc;
            uc = up1;
            up1 = up2;
        }
        wave_sync();
        store_tile(t0);
    }
    const T sc = kk * (acc + ag * yp);

    // backward sweep over the same tiles in reverse, in place in Y (the
    // forward's stores by other lanes of this wave are complete first)
    T yn = T(0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    fetch(Y, (ntiles - 1) * RT, false);
    for (int64_t t = ntiles - 1; t >= 0; --t) {
        const int64_t t0 = t * RT;
        wave_sync();
        put(false);
        wave_sync();
        T v[RT];
        const T *mine = tin + lane * LD;
#pragma unroll
        for (int c = 0; c < RT; ++c) v[c] = mine[c];
        if (t > 0) fetch(Y, t0 - RT, false);
        T cc[RT], cz[RT];
#pragma unroll
        for (int c = 0; c < RT; ++c) {
            cc[c] = t0 + c == n - 1 ? T(0) : cp[t0 + c];
            cz[c] = z[t0 + c];
        }
#pragma unroll
        for (int c = RT - 1; c >= 0; --c) {
            yn = v[c] - cc[c] * yn;
            tout[lane * LD + c] = yn - sc * cz[c];
        }
        wave_sync();
        store_tile(t0);
    }
}

// ---------------------------------------------------------------------------
// Single-pass sweep.  A_c = tridiag(alpha, 1, alpha) with periodic corners is
// circulant and, for |alpha| < 1/2, factors as
//     A_c = c (I + rho S)(I + rho S^T),  rho = (1 - sqrt(1 - 4 alpha^2)) / (2 alpha),
//     c = 1 / (1 + rho^2),  (S y)_j = y_{j+1} (indices mod n),
// so A_c y = d is a cyclic forward recursion f_j = d_j - rho f_{j-1} followed
// by a cyclic backward recursion g_j = f_j - rho g_{j+1}, y = (1 + rho^2) g.
// |rho| < 1 (diagonal dominance, the premise of Sec. 4.2's DistD2): a value
// K steps back (or ahead) enters with weight rho^K, below the rounding unit
// for K >= KT, so each recursion starts K points early from zero and every
// output needs the input only up to K points away.  One read of X and one
// write of Y per point, no intermediate in memory.
// ---------------------------------------------------------------------------
struct OnePassArgs {
    int64_t n, stride, nfib, i3, s12;
    int mode;
    double ca, cb, rho, scale;   // a / (2h), b / (4h), rho, 1 + rho^2
};

// Modes 1 and 2: one lane per fiber (neighbouring lanes read neighbouring
// addresses at every step).  The forward recursion runs K + L points ahead of
// the outputs in a register window F[K + L]; every L points the backward
// recursion runs over the window from its far end and the first L values are
// stored.  The stencil reads of a block are issued before its recursion.  The
// warm-up reads the K + 4 points before point 0 (cyclically); the window past
// the fiber's end reuses f_0 .. f_{K-1} kept in registers, so a fiber is read
// n + K + 8 times.
template <typename T, int K, int L>
__global__ void __launch_bounds__(256) k_compact_lines(const OnePassArgs a, const T *__restrict__ X,
                                                       T *__restrict__ Y) {
    const int64_t n = a.n, s = a.stride;
    const T ca = T(a.ca), cb = T(a.cb), rho = T(a.rho), scale = T(a.scale);
    for (int64_t f = int64_t(blockIdx.x) * 256 + threadIdx.x; f < a.nfib; f += int64_t(gridDim.x) * 256) {
        const int64_t base = a.mode == 1 ? f : (f / a.i3) * a.s12 + f % a.i3;
        const T *u = X + base;
        T *y = Y + base;
        // the stencil stream: point j needs u_{j-2} .. u_{j+2} (mod n); jn is
        // the index (mod n) of the next value to read
        int64_t jn = n - K + 2;
        T um2 = u[(n - K - 2) * s], um1 = u[(n - K - 1) * s], uc = u[(n - K) * s], up1 = u[(n - K + 1) * s];
        auto next_index = [&]() __attribute__((always_inline)) {
            const int64_t j = jn;
            jn = jn + 1 == n ? 0 : jn + 1;
            return j;
        };
        auto step = [&](T up2) __attribute__((always_inline)) {
            const T d = ca * (up1 - um1) + cb * (up2 - um2);
            um2 = um1;
            um1 = uc;
            uc = up1;
            up1 = up2;
            return d;
        };
        // the backward recursion over the window from its far end; the first
        // L values are the outputs of points b .. b + L - 1; then the window
        // moves on by L
        auto emit = [&](T (&W)[K + L], int64_t b0) __attribute__((always_inline)) {
            T g = T(0);
#pragma unroll
            for (int i = K + L - 1; i >= L; --i) g = W[i] - rho * g;
            T out[L];
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                g = W[i] - rho * g;
                out[i] = scale * g;
            }
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (b0 + i < n) y[(b0 + i) * s] = out[i];
#pragma unroll
            for (int i = 0; i < K; ++i) W[i] = W[i + L];
        };
        // forward warm-up over the K points before point 0
        T fprev = T(0);
#pragma unroll 8
        for (int t = 0; t < K; ++t) fprev = step(u[next_index() * s]) - rho * fprev;
        // F[i] = f_{b + i}: first f_0 .. f_{K-1}, kept (fs) for the window
        // past the fiber's end (f is cyclic: f_{n + i} = f_i), so the last
        // blocks read nothing again
        T F[K + L], fs[K];
#pragma unroll
        for (int t = 0; t < K; ++t) {
            fprev = step(u[next_index() * s]) - rho * fprev;
            F[t] = fprev;
            fs[t] = fprev;
        }
        // n and K are multiples of L (host): the last K / L blocks take the
        // whole new part of their window from fs
        static_assert(K % L == 0, "window blocks");
        int64_t b = 0;
        for (; b + K + L <= n; b += L) {
            T v[L];
#pragma unroll
            for (int t = 0; t < L; ++t) v[t] = u[next_index() * s];
#pragma unroll
            for (int t = 0; t < L; ++t) {
                fprev = step(v[t]) - rho * fprev;
                F[K + t] = fprev;
            }
            emit(F, b);
        }
#pragma unroll
        for (int m = 0; m < K / L; ++m, b += L) {
#pragma unroll
            for (int t = 0; t < L; ++t) F[K + t] = fs[m * L + t];
            emit(F, b);
        }
    }
}

// Mode 3: fibers are contiguous rows.  A wave takes one row at a time: the row
// comes into LDS with coalesced 16-byte loads (word l of each 64-word group),
// lane l computes points [c l, c l + c) (c = n / 64): the forward recursion
// from K points before its range, its f values to LDS; then the backward
// recursion from K points past its range over the f values of the lanes
// after it, its y values to LDS; the row leaves with coalesced stores.  Row
// positions are padded by one element every c (lane ranges start in
// different banks).  The next row's words are loaded while a row is
// computed.
// Rows of n = 64 C points, C a power of two, n <= 256 VE (at most four
// 16-byte words per lane); the recursions are unrolled.
template <typename T, int K, int C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_compact_rows1p(const OnePassArgs a, const T *__restrict__ X,
                                                        T *__restrict__ Y) {
    constexpr int VE = 16 / int(sizeof(T)), WPL = 4;
    constexpr int lc = C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : C == 8 ? 3 : 4;
    static_assert((1 << lc) == C && 64 * C <= 256 * VE, "row length");
    extern __shared__ __align__(16) unsigned char smem_1p[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    constexpr int n = 64 * C, c = C, nw = n / VE;
    constexpr int padded = n + 64;
    T *ub = reinterpret_cast<T *>(smem_1p) + wave * 2 * padded;
    T *fb = ub + padded;
    auto pos = [&](int j) __attribute__((always_inline)) { return j + (j >> lc); };
    const T ca = T(a.ca), cb = T(a.cb), rho = T(a.rho), scale = T(a.scale);
    const int64_t wstride = int64_t(gridDim.x) * 4;
    int64_t r = int64_t(blockIdx.x) * 4 + wave;
    V16 buf[WPL];
    auto fetch = [&](int64_t row) __attribute__((always_inline)) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(X + row * n);
#pragma unroll
        for (int i = 0; i < WPL; ++i)
            if (lane + 64 * i < nw) buf[i].u = __builtin_nontemporal_load(src + lane + 64 * i);
    };
    if (r < a.nfib) fetch(r);
    for (; r < a.nfib; r += wstride) {
        wave_sync();
#pragma unroll
        for (int i = 0; i < WPL; ++i)
            if (lane + 64 * i < nw) {
                const int j0 = (lane + 64 * i) * VE;
#pragma unroll
                for (int e = 0; e < VE; ++e) ub[pos(j0 + e)] = reinterpret_cast<const T *>(&buf[i])[e];
            }
        if (r + wstride < a.nfib) fetch(r + wstride);
        wave_sync();
        const int j0 = c * lane;
        // forward: from K points before this lane's range (mod n)
        {
            int j = j0 - K;
            auto U = [&](int k) __attribute__((always_inline)) {   // k in [-K - 2, n + 1]
                const int m = k < 0 ? k + n : (k >= n ? k - n : k);
                return ub[pos(m)];
            };
            T um2 = U(j - 2), um1 = U(j - 1), uc = U(j), up1 = U(j + 1);
            T f = T(0);
#pragma unroll
            for (int t = 0; t < K + c; ++t, ++j) {
                const T up2 = U(j + 2);
                f = ca * (up1 - um1) + cb * (up2 - um2) - rho * f;
                um2 = um1;
                um1 = uc;
                uc = up1;
                up1 = up2;
                if (t >= K) fb[pos(j)] = f;
            }
        }
        wave_sync();
        // backward: from K points past this lane's range (mod n); y overwrites u
        {
            T g = T(0);
#pragma unroll
            for (int t = K + c - 1; t >= 0; --t) {
                int m = j0 + t;
                if (m >= n) m -= n;
                g = fb[pos(m)] - rho * g;
                if (t < c) ub[pos(m)] = scale * g;
            }
        }
        wave_sync();
        u32x4 *dst = reinterpret_cast<u32x4 *>(Y + r * n);
#pragma unroll
        for (int i = 0; i < WPL; ++i)
            if (lane + 64 * i < nw) {
                const int jw = (lane + 64 * i) * VE;
                V16 v;
#pragma unroll
                for (int e = 0; e < VE; ++e) reinterpret_cast<T *>(&v)[e] = ub[pos(jw + e)];
                __builtin_nontemporal_store(v.u, dst + lane + 64 * i);
            }
    }
}

}  // namespace

}  // namespace ttm

using namespace ttm;

extern "C" {

size_t ttm_compact_workspace_size(int64_t n, int dtype) {
    const size_t es = dtype_size(dtype);
    if (n < 3 || (dtype != TTM_F64 && dtype != TTM_F32)) return 0;
    return (size_t(4 * n + 2) * es + 255) & ~size_t(255);
}

int ttm_compact_apply(const int64_t *dims, int mode, const void *X, void *Y, int dtype, const ttm_compact_coef *coef,
                      void *ws, size_t ws_bytes, int prepared, void *stream) {
    if (!dims || !X || !Y || !coef) return TTM_ERR_INVALID_ARG;
    if (mode < 1 || mode > 3) return TTM_ERR_INVALID_ARG;
    if (dtype != TTM_F64 && dtype != TTM_F32) return TTM_ERR_UNSUPPORTED;
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
        if (dims[k] < 1) return TTM_ERR_INVALID_ARG;
        total = checked_prod(total, dims[k]);
        if (total < 0) return TTM_ERR_INVALID_ARG;
    }
    const int64_t n = dims[mode - 1];
    if (n < 3) return TTM_ERR_UNSUPPORTED;
    if (!(coef->h != 0.0) || !isfinite(coef->h) || !isfinite(coef->alpha) || !isfinite(coef->a) ||
        !isfinite(coef->b) || !(fabs(coef->alpha) < 0.5))
        return TTM_ERR_INVALID_ARG;
    const size_t es = dtype_size(dtype);
    if (!aligned(X, es) || !aligned(Y, es)) return TTM_ERR_INVALID_ARG;
    if (overlaps(X, size_t(total) * es, Y, size_t(total) * es)) return TTM_ERR_ALIAS;
    const size_t need = ttm_compact_workspace_size(n, dtype);
    if (!ws || ws_bytes < need || !aligned(ws, 16)) return TTM_ERR_WORKSPACE;
    if (overlaps(ws, need, Y, size_t(total) * es) || overlaps(ws, need, X, size_t(total) * es))
        return TTM_ERR_ALIAS;

    CompactArgs a;
    a.n = n;
    a.mode = mode;
    a.stride = mode == 1 ? dims[1] * dims[2] : (mode == 2 ? dims[2] : 1);
    a.nfib = total / n;
    a.i3 = dims[2];
    a.s12 = dims[1] * dims[2];
    a.ca = coef->a / (2.0 * coef->h);
    a.cb = coef->b / (4.0 * coef->h);
    a.alpha = coef->alpha;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned blocks = unsigned(ceil_div(a.nfib, 256));
    // mode 3: 4 waves of 64 rows per block, each wave with its own LDS tiles
    const unsigned row_blocks = unsigned(ceil_div(a.nfib, 256));
    const size_t prep_lds = n <= COMPACT_PREP_LDS_MAX ? size_t(16 * n) : 0;
    {
        static std::atomic<uint64_t> prep_attr[2];
        const int k = dtype == TTM_F64 ? 0 : 1;
        const void *fn = dtype == TTM_F64 ? reinterpret_cast<const void *>(&k_compact_prep<double>)
                                          : reinterpret_cast<const void *>(&k_compact_prep<float>);
        if (int rc = ensure_lds_limit(fn, size_t(16 * COMPACT_PREP_LDS_MAX), prep_attr[k])) return rc;
    }
    // mode 3: whole tiles take the prefetching kernel
    const bool full_tiles = n % (dtype == TTM_F64 ? RowsCfg<double>::RT : RowsCfg<float>::RT) == 0;
    if (mode == 3) {
        static std::atomic<uint64_t> attr_set[2][2];
        const int k = dtype == TTM_F64 ? 0 : 1, f = full_tiles ? 1 : 0;
        const void *fn = dtype == TTM_F64
                             ? (full_tiles ? reinterpret_cast<const void *>(&k_compact_rows_full<double>)
                                           : reinterpret_cast<const void *>(&k_compact_rows<double>))
                             : (full_tiles ? reinterpret_cast<const void *>(&k_compact_rows_full<float>)
                                           : reinterpret_cast<const void *>(&k_compact_rows<float>));
        const size_t bytes = dtype == TTM_F64 ? 4 * RowsCfg<double>::WAVE_ELEMS * sizeof(double)
                                              : 4 * RowsCfg<float>::WAVE_ELEMS * sizeof(float);
        if (int rc = ensure_lds_limit(fn, bytes, attr_set[k][f])) return rc;
    }
    int rc = TTM_OK;
    // single pass where the recursions' truncation is below the rounding unit
    // (coefficients for the exact sweeps are still prepared when asked, so a
    // later prepared call may take either path)
    const int KT = dtype == TTM_F64 ? 40 : 24;
    const double alpha = coef->alpha;
    const double rho = alpha == 0.0 ? 0.0 : (1.0 - sqrt(1.0 - 4.0 * alpha * alpha)) / (2.0 * alpha);
    const double unit = dtype == TTM_F64 ? 0x1p-53 : 0x1p-24;
    bool onepass = pow(fabs(rho), double(KT)) <= 0.5 * unit && n >= 2 * KT && n % 8 == 0;
    int lc = 0;
    if (mode == 3) {
        const int64_t VE = int64_t(16 / es);
        while ((int64_t(64) << lc) < n) ++lc;
        onepass = onepass && n == (int64_t(64) << lc) && n <= 256 * VE && aligned(X, 16) && aligned(Y, 16);
    }
    OnePassArgs oa;
    oa.n = n;
    oa.stride = a.stride;
    oa.nfib = a.nfib;
    oa.i3 = a.i3;
    oa.s12 = a.s12;
    oa.mode = mode;
    oa.ca = a.ca;
    oa.cb = a.cb;
    oa.rho = rho;
    oa.scale = 1.0 + rho * rho;
    const size_t lds1p = 4 * 2 * size_t(n + 64) * es;
    const unsigned blocks1p = unsigned(std::min<int64_t>(ceil_div(a.nfib, 4), int64_t(device_cu_count()) * 4));
    if (dtype == TTM_F64) {
        if (!prepared)
            rc = launch("ttm_compact_prep", st, [&] {
                hipLaunchKernelGGL(k_compact_prep<double>, dim3(1), dim3(64), prep_lds, st, n, coef->alpha,
                                   static_cast<double *>(ws));
            });
        if (rc == TTM_OK && onepass && mode == 3)
            rc = launch("ttm_compact", st, [&] {
                auto args = [&](auto kern) {
                    hipLaunchKernelGGL(kern, dim3(blocks1p), dim3(256), lds1p, st, oa, static_cast<const double *>(X),
                                       static_cast<double *>(Y));
                };
                switch (lc) {
                    case 0: args(k_compact_rows1p<double, 40, 1>); break;
                    case 1: args(k_compact_rows1p<double, 40, 2>); break;
                    case 2: args(k_compact_rows1p<double, 40, 4>); break;
                    default: args(k_compact_rows1p<double, 40, 8>); break;
                }
            });
        else if (rc == TTM_OK && onepass)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL((k_compact_lines<double, 40, 8>), dim3(blocks), dim3(256), 0, st, oa,
                                   static_cast<const double *>(X), static_cast<double *>(Y));
            });
        else if (rc == TTM_OK && mode == 3)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL(full_tiles ? k_compact_rows_full<double> : k_compact_rows<double>, dim3(row_blocks), dim3(256),
                                   4 * RowsCfg<double>::WAVE_ELEMS * sizeof(double), st, a,
                                   static_cast<const double *>(X), static_cast<double *>(Y),
                                   static_cast<const double *>(ws));
            });
        else if (rc == TTM_OK)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL(k_compact<double>, dim3(blocks), dim3(256), 0, st, a, static_cast<const double *>(X),
                                   static_cast<double *>(Y), static_cast<const double *>(ws));
            });
    } else {
        if (!prepared)
            rc = launch("ttm_compact_prep", st, [&] {
                hipLaunchKernelGGL(k_compact_prep<float>, dim3(1), dim3(64), prep_lds, st, n, coef->alpha,
                                   static_cast<float *>(ws));
            });
        if (rc == TTM_OK && onepass && mode == 3)
            rc = launch("ttm_compact", st, [&] {
                auto args = [&](auto kern) {
                    hipLaunchKernelGGL(kern, dim3(blocks1p), dim3(256), lds1p, st, oa, static_cast<const float *>(X),
                                       static_cast<float *>(Y));
                };
                switch (lc) {
                    case 0: args(k_compact_rows1p<float, 24, 1>); break;
                    case 1: args(k_compact_rows1p<float, 24, 2>); break;
                    case 2: args(k_compact_rows1p<float, 24, 4>); break;
                    case 3: args(k_compact_rows1p<float, 24, 8>); break;
                    default: args(k_compact_rows1p<float, 24, 16>); break;
                }
            });
        else if (rc == TTM_OK && onepass)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL((k_compact_lines<float, 24, 8>), dim3(blocks), dim3(256), 0, st, oa,
                                   static_cast<const float *>(X), static_cast<float *>(Y));
            });
        else if (rc == TTM_OK && mode == 3)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL(full_tiles ? k_compact_rows_full<float> : k_compact_rows<float>, dim3(row_blocks), dim3(256),
                                   4 * RowsCfg<float>::WAVE_ELEMS * sizeof(float), st, a,
                                   static_cast<const float *>(X), static_cast<float *>(Y),
                                   static_cast<const float *>(ws));
            });
        else if (rc == TTM_OK)
            rc = launch("ttm_compact", st, [&] {
                hipLaunchKernelGGL(k_compact<float>, dim3(blocks), dim3(256), 0, st, a, static_cast<const float *>(X),
                                   static_cast<float *>(Y), static_cast<const float *>(ws));
            });
    }
    return rc;
}

}  // extern "C"
