/*
 * ttm_oracle.c -- FP64 reference for the multilinear chain Y = X x1 A x2 B x3 C.
 *
 * TEST INFRASTRUCTURE.  This file is the slow, plain checker the HIP library is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header or constant with
 * the GPU library and the GPU library never calls it.
 *
 * Operator (standard multilinear algebra; the paper applies a 1D operator along
 * one direction of a 3D field, which is a single mode product, Sec. 4.2 Eq.
 * (cfds) with the dense matrix D = A_c^-1 B_c):
 *
 *   (X x_n U)[.., j_n, ..] = sum_{i_n} U[j_n, i_n] * X[.., i_n, ..]
 *   Y[j1,j2,j3] = sum_{i1,i2,i3} A[j1,i1] B[j2,i2] C[j3,i3] X[i1,i2,i3]
 *
 * Storage: every tensor is row-major (C order).  X is [I1][I2][I3] (i3 fastest),
 * a factor U for mode n is [J_n][I_n], Y is [J1][J2][J3].
 *
 * Arithmetic: every value is converted to double on read; each output element
 * is a sequential sum in ascending order of the contracted index.  OpenMP splits
 * only the outermost output index, so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int ttmo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * One mode product.  dims = (I1, I2, I3) of the input, Jn replaces dims[mode-1].
 * Two readers: a double input and a float input (exact upcast).
 * ------------------------------------------------------------------------- */
#define DEFINE_MODE_PRODUCT(NAME, XT)                                              \
void NAME(int mode, const int64_t *dims, int64_t Jn, const XT *X,                 \
          const double *U, double *Out)                                            \
{                                                                                  \
    const int64_t n1 = dims[0], n2 = dims[1], n3 = dims[2];                        \
    if (mode == 1) {                                                               \
        /* Out[j1][i2][i3] = sum_i1 U[j1][i1] X[i1][i2][i3]; the sum over i1 for   \
           every (i2,i3) is accumulated in ascending i1 order. */                  \
        const int64_t plane = n2 * n3;                                             \
        _Pragma("omp parallel for schedule(static)")                               \
        for (int64_t j = 0; j < Jn; ++j) {                                         \
            double *o = Out + j * plane;                                           \
            for (int64_t p = 0; p < plane; ++p) o[p] = 0.0;                        \
            for (int64_t i = 0; i < n1; ++i) {                                     \
                const double u = U[j * n1 + i];                                    \
                const XT *x = X + i * plane;                                       \
                for (int64_t p = 0; p < plane; ++p) o[p] += u * (double)x[p];      \
            }                                                                      \
        }                                                                          \
    } else if (mode == 2) {                                                        \
        /* Out[i1][j2][i3] = sum_i2 U[j2][i2] X[i1][i2][i3] */                     \
        _Pragma("omp parallel for schedule(static)")                               \
        for (int64_t a = 0; a < n1; ++a) {                                         \
            for (int64_t j = 0; j < Jn; ++j) {                                     \
                double *o = Out + (a * Jn + j) * n3;                               \
                for (int64_t c = 0; c < n3; ++c) o[c] = 0.0;                       \
                for (int64_t i = 0; i < n2; ++i) {                                 \
                    const double u = U[j * n2 + i];                                \
                    const XT *x = X + (a * n2 + i) * n3;                           \
                    for (int64_t c = 0; c < n3; ++c) o[c] += u * (double)x[c];     \
                }                                                                  \
            }                                                                      \
        }                                                                          \
    } else {                                                                       \
        /* Out[i1][i2][j3] = sum_i3 U[j3][i3] X[i1][i2][i3] */                     \
        _Pragma("omp parallel for schedule(static)")                               \
        for (int64_t a = 0; a < n1; ++a) {                                         \
            for (int64_t b = 0; b < n2; ++b) {                                     \
                const XT *x = X + (a * n2 + b) * n3;                               \
                double *o = Out + (a * n2 + b) * Jn;                               \
                for (int64_t j = 0; j < Jn; ++j) {                                 \
                    double s = 0.0;                                                \
                    for (int64_t i = 0; i < n3; ++i)                               \
                        s += U[j * n3 + i] * (double)x[i];                         \
                    o[j] = s;                                                      \
                }                                                                  \
            }                                                                      \
        }                                                                          \
    }                                                                              \
}

DEFINE_MODE_PRODUCT(ttmo_mode_product, double)
DEFINE_MODE_PRODUCT(ttmo_mode_product_xf32, float)

/* ---------------------------------------------------------------------------
 * The chain, applying the three mode products in a caller-chosen order
 * (order[k] in {1,2,3}, a permutation).  The mode products for distinct modes
 * commute, so every order is the same operator; the default order is 1,2,3 as
 * the chain is written.  Intermediates are double.
 * ------------------------------------------------------------------------- */
static int chain_ordered_impl(const int *order, const int64_t *I, const int64_t *J,
                              const double *Xd, const float *Xf,
                              const double *A, const double *B, const double *C,
                              double *Y)
{
    const double *U[3] = {A, B, C};
    int64_t dims[3] = {I[0], I[1], I[2]};
    double *cur = NULL;
    for (int step = 0; step < 3; ++step) {
        const int m = order[step];
        if (m < 1 || m > 3) { free(cur); return -1; }
        int64_t out_dims[3] = {dims[0], dims[1], dims[2]};
        out_dims[m - 1] = J[m - 1];
        const int64_t n_out = out_dims[0] * out_dims[1] * out_dims[2];
        double *nxt = (step == 2) ? Y : (double *)malloc(sizeof(double) * (size_t)(n_out > 0 ? n_out : 1));
        if (!nxt) { free(cur); return -2; }
        if (step == 0 && Xf)
            ttmo_mode_product_xf32(m, dims, J[m - 1], Xf, U[m - 1], nxt);
        else
            ttmo_mode_product(m, dims, J[m - 1], step == 0 ? Xd : cur, U[m - 1], nxt);
        if (step > 0) free(cur);
        cur = nxt;
        memcpy(dims, out_dims, sizeof dims);
    }
    return 0;
}

int ttmo_chain_ordered(const int *order, const int64_t *I, const int64_t *J,
                       const double *X, const double *A, const double *B,
                       const double *C, double *Y)
{
    return chain_ordered_impl(order, I, J, X, NULL, A, B, C, Y);
}

int ttmo_chain_ordered_xf32(const int *order, const int64_t *I, const int64_t *J,
                            const float *X, const double *A, const double *B,
                            const double *C, double *Y)
{
    return chain_ordered_impl(order, I, J, NULL, X, A, B, C, Y);
}

int ttmo_chain(const int64_t *I, const int64_t *J, const double *X, const double *A,
               const double *B, const double *C, double *Y)
{
    static const int order[3] = {1, 2, 3};
    return chain_ordered_impl(order, I, J, X, NULL, A, B, C, Y);
}

/* The definition written out: a six-fold sum per output element (tiny shapes). */
void ttmo_brute(const int64_t *I, const int64_t *J, const double *X, const double *A,
                const double *B, const double *C, double *Y)
{
    for (int64_t j1 = 0; j1 < J[0]; ++j1)
    for (int64_t j2 = 0; j2 < J[1]; ++j2)
    for (int64_t j3 = 0; j3 < J[2]; ++j3) {
        double s = 0.0;
        for (int64_t i1 = 0; i1 < I[0]; ++i1)
        for (int64_t i2 = 0; i2 < I[1]; ++i2)
        for (int64_t i3 = 0; i3 < I[2]; ++i3)
            s += A[j1 * I[0] + i1] * B[j2 * I[1] + i2] * C[j3 * I[2] + i3]
               * X[(i1 * I[1] + i2) * I[2] + i3];
        Y[(j1 * J[1] + j2) * J[2] + j3] = s;
    }
}

/* ---------------------------------------------------------------------------
 * Loss and gradients for L = 1/2 ||Y - T||_F^2 with G = dL/dY = Y - T.
 *   dX = G x1 A^T x2 B^T x3 C^T
 *   dA[j1,i1] = sum_{j2,j3} G[j1,j2,j3] (X x2 B x3 C)[i1,j2,j3]
 *   dB[j2,i2] = sum_{j1,j3} G[j1,j2,j3] (X x1 A x3 C)[j1,i2,j3]
 *   dC[j3,i3] = sum_{j1,j2} G[j1,j2,j3] (X x1 A x2 B)[j1,j2,i3]
 * Any of dX, dA, dB, dC may be NULL.
 * ------------------------------------------------------------------------- */
static double *transpose(const double *U, int64_t rows, int64_t cols)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)(rows * cols > 0 ? rows * cols : 1));
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c)
            t[c * rows + r] = U[r * cols + c];
    return t;
}

double ttmo_loss(const int64_t *I, const int64_t *J, const double *X, const double *A,
                 const double *B, const double *C, const double *T)
{
    const int64_t ny = J[0] * J[1] * J[2];
    double *Y = (double *)malloc(sizeof(double) * (size_t)ny);
    ttmo_chain(I, J, X, A, B, C, Y);
    double s = 0.0;
    for (int64_t k = 0; k < ny; ++k) {
        const double r = Y[k] - T[k];
        s += r * r;
    }
    free(Y);
    return 0.5 * s;
}

int ttmo_backward(const int64_t *I, const int64_t *J, const double *G, const double *X,
                  const double *A, const double *B, const double *C,
                  double *dX, double *dA, double *dB, double *dC)
{
    if (dX) {
        /* transposed factors map J_n back to I_n */
        double *At = transpose(A, J[0], I[0]);
        double *Bt = transpose(B, J[1], I[1]);
        double *Ct = transpose(C, J[2], I[2]);
        int rc = ttmo_chain(J, I, G, At, Bt, Ct, dX);
        free(At); free(Bt); free(Ct);
        if (rc) return rc;
    }
    if (dA) {
        static const int ord[3] = {2, 3, 1};   /* Z = X x2 B x3 C: [I1][J2][J3] */
        int64_t Jz[3] = {I[0], J[1], J[2]};
        double *eye = (double *)calloc((size_t)(I[0] * I[0]), sizeof(double));
        for (int64_t k = 0; k < I[0]; ++k) eye[k * I[0] + k] = 1.0;
        double *Z = (double *)malloc(sizeof(double) * (size_t)(I[0] * J[1] * J[2]));
        chain_ordered_impl(ord, I, Jz, X, NULL, eye, B, C, Z);
        for (int64_t j1 = 0; j1 < J[0]; ++j1)
            for (int64_t i1 = 0; i1 < I[0]; ++i1) {
                double s = 0.0;
                for (int64_t j2 = 0; j2 < J[1]; ++j2)
                    for (int64_t j3 = 0; j3 < J[2]; ++j3)
                        s += G[(j1 * J[1] + j2) * J[2] + j3] * Z[(i1 * J[1] + j2) * J[2] + j3];
                dA[j1 * I[0] + i1] = s;
            }
        free(Z); free(eye);
    }
    if (dB) {
        static const int ord[3] = {1, 3, 2};   /* Z = X x1 A x3 C: [J1][I2][J3] */
        int64_t Jz[3] = {J[0], I[1], J[2]};
        double *eye = (double *)calloc((size_t)(I[1] * I[1]), sizeof(double));
        for (int64_t k = 0; k < I[1]; ++k) eye[k * I[1] + k] = 1.0;
        double *Z = (double *)malloc(sizeof(double) * (size_t)(J[0] * I[1] * J[2]));
        chain_ordered_impl(ord, I, Jz, X, NULL, A, eye, C, Z);
        for (int64_t j2 = 0; j2 < J[1]; ++j2)
            for (int64_t i2 = 0; i2 < I[1]; ++i2) {
                double s = 0.0;
                for (int64_t j1 = 0; j1 < J[0]; ++j1)
                    for (int64_t j3 = 0; j3 < J[2]; ++j3)
                        s += G[(j1 * J[1] + j2) * J[2] + j3] * Z[(j1 * I[1] + i2) * J[2] + j3];
                dB[j2 * I[1] + i2] = s;
            }
        free(Z); free(eye);
    }
    if (dC) {
        static const int ord[3] = {1, 2, 3};   /* Z = X x1 A x2 B: [J1][J2][I3] */
        int64_t Jz[3] = {J[0], J[1], I[2]};
        double *eye = (double *)calloc((size_t)(I[2] * I[2]), sizeof(double));
        for (int64_t k = 0; k < I[2]; ++k) eye[k * I[2] + k] = 1.0;
        double *Z = (double *)malloc(sizeof(double) * (size_t)(J[0] * J[1] * I[2]));
        chain_ordered_impl(ord, I, Jz, X, NULL, A, B, eye, Z);
        for (int64_t j3 = 0; j3 < J[2]; ++j3)
            for (int64_t i3 = 0; i3 < I[2]; ++i3) {
                double s = 0.0;
                for (int64_t j1 = 0; j1 < J[0]; ++j1)
                    for (int64_t j2 = 0; j2 < J[1]; ++j2)
                        s += G[(j1 * J[1] + j2) * J[2] + j3] * Z[(j1 * J[1] + j2) * I[2] + i3];
                dC[j3 * I[2] + i3] = s;
            }
        free(Z); free(eye);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Batched chain over independent cuboids stored back to back.
 * dims is count x 6: (I1, I2, I3, J1, J2, J3) per cuboid.  Cuboid k's X, A, B,
 * C and Y start where cuboid k-1's end (running sums of the element counts).
 * ------------------------------------------------------------------------- */
int ttmo_batched(int64_t count, const int64_t *dims, const double *X, const double *A,
                 const double *B, const double *C, double *Y)
{
    int64_t ox = 0, oa = 0, ob = 0, oc = 0, oy = 0;
    for (int64_t k = 0; k < count; ++k) {
        const int64_t *d = dims + 6 * k;
        const int64_t I[3] = {d[0], d[1], d[2]};
        const int64_t J[3] = {d[3], d[4], d[5]};
        int rc = ttmo_chain(I, J, X + ox, A + oa, B + ob, C + oc, Y + oy);
        if (rc) return rc;
        ox += I[0] * I[1] * I[2];
        oa += J[0] * I[0];
        ob += J[1] * I[1];
        oc += J[2] * I[2];
        oy += J[0] * J[1] * J[2];
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * One tridiagonal system T u = d (Sec. 2.1: the Thomas algorithm is Gaussian
 * elimination without pivoting specialised to the band).  a = lower band
 * (a[0] unused), b = diagonal, c = upper band (c[n-1] unused).
 *
 * Written here as an explicit factorisation T = L U and two substitutions:
 *   L is unit lower bidiagonal with sub-diagonal m[i] (row i, column i-1),
 *   U is upper bidiagonal with diagonal p[i] and the unchanged super-diagonal
 *   c, so row i of L U gives a[i] = m[i] p[i-1] and b[i] = m[i] c[i-1] + p[i].
 * Then L y = d (forward) and U u = y (backward).
 * ------------------------------------------------------------------------- */
static void tri_lu(int64_t n, const double *a, const double *b, const double *c, double *m, double *p)
{
    p[0] = b[0];
    m[0] = 0.0;
    for (int64_t i = 1; i < n; ++i) {
        m[i] = a[i] / p[i - 1];
        p[i] = b[i] - m[i] * c[i - 1];
    }
}

/* L y = d with L = I + (sub-diagonal m) */
static void tri_forward(int64_t n, const double *m, const double *d, double *y)
{
    y[0] = d[0];
    for (int64_t i = 1; i < n; ++i) y[i] = d[i] - m[i] * y[i - 1];
}

/* U u = y with U = diag(p) + (super-diagonal c) */
static void tri_backward(int64_t n, const double *p, const double *c, const double *y, double *u)
{
    u[n - 1] = y[n - 1] / p[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) u[i] = (y[i] - c[i] * u[i + 1]) / p[i];
}

int ttmo_thomas(int64_t n, const double *a, const double *b, const double *c,
                const double *d, double *u)
{
    if (n < 1) return -1;
    double *m = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    tri_lu(n, a, b, c, m, p);
    tri_forward(n, m, d, y);
    tri_backward(n, p, c, y, u);
    free(m); free(p); free(y);
    return 0;
}

/* Cyclic tridiagonal system (corner entries a[0] at (0,n-1) and c[n-1] at
 * (n-1,0)) by the Sherman-Morrison correction of two Thomas solves, the
 * "periodic Thomas" variant the paper names in Sec. 2.1.  Needs n >= 3. */
int ttmo_thomas_periodic(int64_t n, const double *a, const double *b, const double *c,
                         const double *d, double *u)
{
    if (n < 3) return -1;
    const double gamma = -b[0];
    double *bb = (double *)malloc(sizeof(double) * (size_t)n);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(bb, b, sizeof(double) * (size_t)n);
    bb[0] = b[0] - gamma;
    bb[n - 1] = b[n - 1] - c[n - 1] * a[0] / gamma;
    ttmo_thomas(n, a, bb, c, d, u);
    for (int64_t i = 0; i < n; ++i) rhs[i] = 0.0;
    rhs[0] = gamma;
    rhs[n - 1] = c[n - 1];
    ttmo_thomas(n, a, bb, c, rhs, z);
    const double fact = (u[0] + a[0] * u[n - 1] / gamma) / (1.0 + z[0] + a[0] * z[n - 1] / gamma);
    for (int64_t i = 0; i < n; ++i) u[i] -= fact * z[i];
    free(bb); free(rhs); free(z);
    return 0;
}

/* ---------------------------------------------------------------------------
 * The paper's compact sixth-order first derivative (Sec. 4.2, Eq. (cfds)) on
 * a periodic grid, applied along one mode of X: for every fiber u along mode
 * `mode` (length n = dims[mode-1] >= 3, indices taken mod n)
 *
 *   d_i = a (u_{i+1} - u_{i-1}) / (2h) + b (u_{i+2} - u_{i-2}) / (4h)
 *   alpha u'_{i-1} + u'_i + alpha u'_{i+1} = d_i      (cyclic tridiagonal)
 *
 * solved with ttmo_thomas_periodic (Sec. 2.1).  Y has the shape of X.  This is
 * Y = X x_mode D with D = A_c^-1 B_c, without forming D.
 * ------------------------------------------------------------------------- */
int ttmo_compact6_apply(int mode, const int64_t *dims, double alpha, double a, double b, double h,
                        const double *X, double *Y)
{
    if (mode < 1 || mode > 3) return -1;
    const int64_t n = dims[mode - 1];
    if (n < 3) return -1;
    int64_t stride = 1;
    for (int m = mode; m < 3; ++m) stride *= dims[m];
    const int64_t outer = (mode == 1) ? 1 : (mode == 2 ? dims[0] : dims[0] * dims[1]);
    const int64_t inner = stride;                      /* fibers per outer index */
    int rc = 0;
#pragma omp parallel for schedule(static) reduction(|: rc)
    for (int64_t o = 0; o < outer; ++o) {
        double *lo = (double *)malloc(sizeof(double) * (size_t)n);
        double *di = (double *)malloc(sizeof(double) * (size_t)n);
        double *up = (double *)malloc(sizeof(double) * (size_t)n);
        double *u = (double *)malloc(sizeof(double) * (size_t)n);
        double *d = (double *)malloc(sizeof(double) * (size_t)n);
        double *x = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) { lo[i] = alpha; di[i] = 1.0; up[i] = alpha; }
        for (int64_t f = 0; f < inner; ++f) {
            const int64_t base = o * n * stride + f;
            for (int64_t i = 0; i < n; ++i) u[i] = X[base + i * stride];
            for (int64_t i = 0; i < n; ++i) {
                const double up1 = u[(i + 1) % n], um1 = u[(i + n - 1) % n];
                const double up2 = u[(i + 2) % n], um2 = u[(i + n - 2) % n];
                d[i] = a * (up1 - um1) / (2.0 * h) + b * (up2 - um2) / (4.0 * h);
            }
            rc |= ttmo_thomas_periodic(n, lo, di, up, d, x);
            for (int64_t i = 0; i < n; ++i) Y[base + i * stride] = x[i];
        }
        free(lo); free(di); free(up); free(u); free(d); free(x);
    }
    return rc ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Reordering a field between directional layouts (Sec. 4.1: each direction
 * has its own layout, and a reorder moves a field from one to another;
 * Sec. 5.3 counts these moves in the transport equation's data movement).
 * For a 3-way array X of dims (n0, n1, n2) and a permutation perm of
 * {0, 1, 2}, Y's axis k is X's axis perm[k]:
 *   Y[i_perm[0]][i_perm[1]][i_perm[2]] = X[i0][i1][i2],
 * Y of dims (n_perm[0], n_perm[1], n_perm[2]).  Elements are es bytes (4:
 * float, 8: double) and are moved as bytes, so the result is bit-exact.
 * accumulate != 0: Y += that instead (the accumulation of a direction's
 * result into another layout), the sum taken in double and rounded to the
 * element type, which is the correctly rounded sum of the two stored values.
 * ------------------------------------------------------------------------- */
int ttmo_reorder(const int64_t *dims, const int *perm, const void *X, void *Y, int es, int accumulate)
{
    if (es != 4 && es != 8) return -1;
    int seen[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        if (perm[k] < 0 || perm[k] > 2 || seen[perm[k]]) return -1;
        seen[perm[k]] = 1;
    }
    const int64_t yd[3] = {dims[perm[0]], dims[perm[1]], dims[perm[2]]};
    const unsigned char *xb = (const unsigned char *)X;
    unsigned char *yb = (unsigned char *)Y;
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < dims[0]; ++i0) {
        int64_t idx[3];
        idx[0] = i0;
        for (idx[1] = 0; idx[1] < dims[1]; ++idx[1]) {
            for (idx[2] = 0; idx[2] < dims[2]; ++idx[2]) {
                const int64_t src = (idx[0] * dims[1] + idx[1]) * dims[2] + idx[2];
                const int64_t dst = (idx[perm[0]] * yd[1] + idx[perm[1]]) * yd[2] + idx[perm[2]];
                if (!accumulate) {
                    memcpy(yb + dst * es, xb + src * es, (size_t)es);
                } else if (es == 4) {
                    float *y = (float *)(yb + dst * 4);
                    const float x = *(const float *)(xb + src * 4);
                    *y = (float)((double)*y + (double)x);
                } else {
                    double *y = (double *)(yb + dst * 8);
                    *y = *y + *(const double *)(xb + src * 8);
                }
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Gram matrix of a mode-n unfolding, G = X_(n) X_(n)^T (I_n x I_n):
 *   G[a][b] = sum over the other two indices of X[..a..] X[..b..],
 * the matrix whose leading eigenvectors are the leading left singular
 * vectors of X_(n), i.e. the truncated HOSVD factor of mode n.  Sequential
 * sums in ascending order of the other indices (i1 before i2 before i3).
 * ------------------------------------------------------------------------- */
int ttmo_gram(const int64_t *dims, int mode, const double *X, double *G)
{
    if (mode < 1 || mode > 3) return -1;
    const int64_t n1 = dims[0], n2 = dims[1], n3 = dims[2];
    const int64_t n = dims[mode - 1];
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t b = 0; b < n; ++b) {
            double s = 0.0;
            if (mode == 1) {
                for (int64_t j = 0; j < n2; ++j)
                    for (int64_t k = 0; k < n3; ++k) s += X[(a * n2 + j) * n3 + k] * X[(b * n2 + j) * n3 + k];
            } else if (mode == 2) {
                for (int64_t i = 0; i < n1; ++i)
                    for (int64_t k = 0; k < n3; ++k) s += X[(i * n2 + a) * n3 + k] * X[(i * n2 + b) * n3 + k];
            } else {
                for (int64_t i = 0; i < n1; ++i)
                    for (int64_t j = 0; j < n2; ++j) s += X[(i * n2 + j) * n3 + a] * X[(i * n2 + j) * n3 + b];
            }
            G[a * n + b] = s;
        }
    }
    return 0;
}
