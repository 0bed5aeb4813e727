"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, gcc) and driven through every entry point on small ragged shapes,
each buffer allocated to its exact size: an out-of-bounds access, a leak or
undefined behaviour aborts the driver.  The OpenMP pragmas are left out of
this build (the loops run sequentially)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ttm_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void ttmo_mode_product(int mode, const int64_t *dims, int64_t J, const double *X, const double *U, double *Y);
int ttmo_chain(const int64_t *I, const int64_t *J, const double *X, const double *A, const double *B,
               const double *C, double *Y);
int ttmo_chain_ordered(const int *order, const int64_t *I, const int64_t *J, const double *X, const double *A,
                       const double *B, const double *C, double *Y);
int ttmo_chain_ordered_xf32(const int *order, const int64_t *I, const int64_t *J, const float *X, const double *A,
                            const double *B, const double *C, double *Y);
void ttmo_brute(const int64_t *I, const int64_t *J, const double *X, const double *A, const double *B,
                const double *C, double *Y);
double ttmo_loss(const int64_t *I, const int64_t *J, const double *X, const double *A, const double *B,
                 const double *C, const double *T);
int ttmo_backward(const int64_t *I, const int64_t *J, const double *G, const double *X, const double *A,
                  const double *B, const double *C, double *dX, double *dA, double *dB, double *dC);
int ttmo_batched(int64_t count, const int64_t *dims, const double *X, const double *A, const double *B,
                 const double *C, double *Y);
int ttmo_thomas(int64_t n, const double *a, const double *b, const double *c, const double *d, double *u);
int ttmo_thomas_periodic(int64_t n, const double *a, const double *b, const double *c, const double *d,
                         double *u);
int ttmo_compact6_apply(int mode, const int64_t *dims, double alpha, double a, double b, double h,
                        const double *X, double *Y);
int ttmo_reorder(const int64_t *dims, const int *perm, const void *X, void *Y, int es, int accumulate);
int ttmo_gram(const int64_t *dims, int mode, const double *X, double *G);

static double *vec(int64_t n, double seed) {
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = sin(seed + 0.37 * (double)i);
    return p;
}
#define CHECK(x) do { if ((x) != 0) { fprintf(stderr, "failed: %s\n", #x); return 1; } } while (0)

static int chain_case(int64_t i1, int64_t i2, int64_t i3, int64_t j1, int64_t j2, int64_t j3) {
    const int64_t I[3] = {i1, i2, i3}, J[3] = {j1, j2, j3};
    const int64_t nx = i1 * i2 * i3, ny = j1 * j2 * j3;
    double *X = vec(nx, 1), *A = vec(j1 * i1, 2), *B = vec(j2 * i2, 3), *C = vec(j3 * i3, 4);
    double *Y = vec(ny, 0), *Yb = vec(ny, 0), *T = vec(ny, 5);
    float *Xf = (float *)malloc(sizeof(float) * (size_t)nx);
    for (int64_t k = 0; k < nx; ++k) Xf[k] = (float)X[k];
    const int orders[6][3] = {{1, 2, 3}, {1, 3, 2}, {2, 1, 3}, {2, 3, 1}, {3, 1, 2}, {3, 2, 1}};
    CHECK(ttmo_chain(I, J, X, A, B, C, Y));
    for (int o = 0; o < 6; ++o) {
        CHECK(ttmo_chain_ordered(orders[o], I, J, X, A, B, C, Y));
        CHECK(ttmo_chain_ordered_xf32(orders[o], I, J, Xf, A, B, C, Y));
    }
    ttmo_brute(I, J, X, A, B, C, Yb);
    (void)ttmo_loss(I, J, X, A, B, C, T);
    double *dX = vec(nx, 0), *dA = vec(j1 * i1, 0), *dB = vec(j2 * i2, 0), *dC = vec(j3 * i3, 0);
    CHECK(ttmo_backward(I, J, T, X, A, B, C, dX, dA, dB, dC));
    CHECK(ttmo_backward(I, J, T, X, A, B, C, NULL, dA, NULL, dC));
    CHECK(ttmo_backward(I, J, T, X, A, B, C, dX, NULL, dB, NULL));
    for (int m = 1; m <= 3; ++m) {
        const int64_t n = I[m - 1];
        double *G = vec(n * n, 0);
        CHECK(ttmo_gram(I, m, X, G));
        free(G);
        const int64_t jm = J[m - 1];
        const int64_t ny1 = nx / n * jm;
        double *Ym = vec(ny1, 0), *U = vec(jm * n, 6);
        ttmo_mode_product(m, I, jm, X, U, Ym);
        free(Ym); free(U);
    }
    free(X); free(A); free(B); free(C); free(Y); free(Yb); free(T); free(Xf);
    free(dX); free(dA); free(dB); free(dC);
    return 0;
}

int main(void) {
    CHECK(chain_case(3, 4, 5, 2, 3, 6));
    CHECK(chain_case(1, 1, 1, 1, 1, 1));
    CHECK(chain_case(5, 1, 3, 1, 4, 2));
    CHECK(chain_case(2, 7, 1, 3, 1, 5));
    /* batched: three cuboids back to back */
    const int64_t dims[18] = {3, 4, 5, 2, 3, 6, 1, 1, 1, 1, 1, 1, 4, 2, 3, 5, 1, 2};
    int64_t nx = 0, na = 0, nb = 0, nc = 0, ny = 0;
    for (int k = 0; k < 3; ++k) {
        const int64_t *d = dims + 6 * k;
        nx += d[0] * d[1] * d[2]; na += d[3] * d[0]; nb += d[4] * d[1]; nc += d[5] * d[2];
        ny += d[3] * d[4] * d[5];
    }
    double *X = vec(nx, 1), *A = vec(na, 2), *B = vec(nb, 3), *C = vec(nc, 4), *Y = vec(ny, 0);
    CHECK(ttmo_batched(3, dims, X, A, B, C, Y));
    free(X); free(A); free(B); free(C); free(Y);
    /* tridiagonal solves, plain and cyclic */
    const int64_t ns[4] = {1, 3, 5, 9};
    for (int t = 0; t < 4; ++t) {
        const int64_t n = ns[t];
        double *a = vec(n, 1), *b = vec(n, 2), *c = vec(n, 3), *d = vec(n, 4), *u = vec(n, 0);
        for (int64_t i = 0; i < n; ++i) b[i] = 4.0 + b[i];
        CHECK(ttmo_thomas(n, a, b, c, d, u));
        if (n >= 3) CHECK(ttmo_thomas_periodic(n, a, b, c, d, u));
        free(a); free(b); free(c); free(d); free(u);
    }
    /* compact operator along each mode, and the reorders */
    const int64_t cd[3] = {3, 4, 5};
    double *Xc = vec(60, 7), *Yc = vec(60, 0);
    for (int m = 1; m <= 3; ++m)
        CHECK(ttmo_compact6_apply(m, cd, 1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0, 0.1, Xc, Yc));
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    float *Xs = (float *)malloc(sizeof(float) * 60), *Ys = (float *)malloc(sizeof(float) * 60);
    for (int k = 0; k < 60; ++k) { Xs[k] = (float)k; Ys[k] = 0.f; }
    for (int p = 0; p < 6; ++p)
        for (int acc = 0; acc < 2; ++acc) {
            CHECK(ttmo_reorder(cd, perms[p], Xc, Yc, 8, acc));
            CHECK(ttmo_reorder(cd, perms[p], Xs, Ys, 4, acc));
        }
    free(Xc); free(Yc); free(Xs); free(Ys);
    printf("oracle under sanitizers: ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behavior_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", SRC, str(drv), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle under sanitizers: ok" in r.stdout
