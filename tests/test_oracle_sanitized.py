"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a small driver calls every entry point on a 2D Poisson matrix,
a matrix with empty rows and random multi-word vectors, in all eight
arithmetics; any out-of-bounds access, leak or undefined operation fails the
run.  The same source, unsanitised and with OpenMP, is what the other
oracle tests load."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <math.h>
typedef struct { int32_t iters, status; double rel_res, seconds; } info_t;
int mwo_eft(int, long, const double *, const double *, double *, double *);
int mwo_elementwise(int, int, long, const double *, const double *, double *);
int mwo_spmv(int, long, const int32_t *, const int32_t *, const double *, const double *, double *);
int mwo_dot(int, long, const double *, const double *, double *);
int mwo_axpy(int, long, const double *, const double *, double *);
int mwo_cg_solve(int, long, const int32_t *, const int32_t *, const double *, const double *, double *, double,
                 int32_t, int32_t, info_t *, double *);
int mwo_pcg_jacobi_solve(int, long, const int32_t *, const int32_t *, const double *, const double *, double *,
                         double, int32_t, int32_t, info_t *, double *);
int mwo_dot_error(int, long, const double *, const double *, const double *, double *, double *);
int mwo_spmv_error(int, long, const int32_t *, const int32_t *, const double *, const double *, const double *,
                   long, const int64_t *, double *, double *);
int mwo_true_residual(int, long, const int32_t *, const int32_t *, const double *, const double *, const double *,
                      double *);

static double rnd(unsigned *s) { *s = *s * 1103515245u + 12345u; return ((*s >> 8) & 0xffff) / 32768.0 - 1.0; }

int main(void)
{
    const int m = 9, n = m * m;             /* 2D Poisson 9 x 9 */
    int32_t *rp = malloc(sizeof(int32_t) * (n + 1)), *ci = malloc(sizeof(int32_t) * 5 * n);
    double *va = malloc(sizeof(double) * 5 * n);
    int nnz = 0;
    for (int i = 0; i < n; ++i) {
        rp[i] = nnz;
        const int r = i / m, c = i % m;
        if (r > 0) { ci[nnz] = i - m; va[nnz++] = -1.0; }
        if (c > 0) { ci[nnz] = i - 1; va[nnz++] = -1.0; }
        ci[nnz] = i; va[nnz++] = 4.0;
        if (c < m - 1) { ci[nnz] = i + 1; va[nnz++] = -1.0; }
        if (r < m - 1) { ci[nnz] = i + m; va[nnz++] = -1.0; }
    }
    rp[n] = nnz;
    /* rows 3 and 7 of a second matrix are empty */
    int32_t rp2[11] = {0, 1, 2, 3, 3, 5, 6, 7, 7, 8, 9}, ci2[9] = {0, 1, 2, 3, 4, 5, 6, 8, 9};
    double va2[9] = {1, 2, 3, 4, 5, 6, 7, 8, 9};
    unsigned seed = 7;
    int bad = 0;
    for (int a = 0; a < 8; ++a) {
        const int k = a == 0 ? 1 : (a < 3 ? 2 : (a < 6 ? 3 : 4));
        double *u = malloc(sizeof(double) * 4 * n), *v = malloc(sizeof(double) * 4 * n);
        double *w = malloc(sizeof(double) * 4 * n), *y = malloc(sizeof(double) * 4 * n);
        double *b = malloc(sizeof(double) * n), *x = calloc(4 * n, sizeof(double)), *hist = malloc(sizeof(double) * 400);
        for (int i = 0; i < 4 * n; ++i) { u[i] = rnd(&seed) * (i < n ? 1.0 : 1e-17); v[i] = rnd(&seed) * (i < n ? 1.0 : 1e-17) + (i < n ? 3.0 : 0.0); }
        for (int i = 0; i < n; ++i) b[i] = rnd(&seed);
        for (int op = 0; op <= 6; ++op) bad |= mwo_elementwise(a, op, n, u, v, w) != 0;
        bad |= mwo_spmv(a, n, rp, ci, va, u, y) != 0;
        bad |= mwo_spmv(a, 10, rp2, ci2, va2, u, y) != 0;
        double res[4], ae, sc;
        bad |= mwo_dot(a, n, u, v, res) != 0;
        bad |= mwo_dot_error(a, n, u, v, res, &ae, &sc) != 0;
        double alpha[4] = {0.5, 1e-17, 1e-34, 1e-51};
        bad |= mwo_axpy(a, n, alpha, u, w) != 0;
        int64_t rows[4] = {0, 5, 40, n - 1};
        double errs[4], scs[4];
        bad |= mwo_spmv_error(a, n, rp, ci, va, u, y, 0, NULL, NULL, NULL) < 0;
        mwo_spmv(a, n, rp, ci, va, u, y);
        bad |= mwo_spmv_error(a, n, rp, ci, va, u, y, 4, rows, errs, scs) != 0;
        info_t info;
        bad |= mwo_cg_solve(a, n, rp, ci, va, b, x, 1e-12, 400, 1, &info, hist) != 0;
        double tr;
        bad |= mwo_true_residual(a, n, rp, ci, va, b, x, &tr) != 0 || !(tr < 1e-9);
        for (int i = 0; i < 4 * n; ++i) x[i] = 0.0;
        bad |= mwo_pcg_jacobi_solve(a, n, rp, ci, va, b, x, 1e-12, 400, 1, &info, hist) != 0;
        for (int i = 0; i < 4 * n; ++i) x[i] = 0.0;
        bad |= mwo_cg_solve(a, n, rp, ci, va, b, x, 0.0, 3, 0, &info, NULL) != 1;   /* maxit, no normalisation */
        free(u); free(v); free(w); free(y); free(b); free(x); free(hist);
        (void)k;
    }
    double e1[4] = {1.0, 1e300, -0.0, 3.0}, e2[4] = {1e-300, 1e300, 0.0, -3.0}, o1[4], o2[4];
    for (int which = 0; which < 3; ++which) bad |= mwo_eft(which, 4, e1, e2, o1, o2) != 0;
    free(rp); free(ci); free(va);
    printf(bad ? "FAILED\n" : "OK\n");
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(exe),
           os.path.join(ROOT, "oracle", "mwo.c"), str(drv), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    # verify_asan_link_order=0: the sanitiser runtime need not be the first
    # library loaded (an environment may preload another one)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "OK", (r.stdout[-2000:], r.stderr[-3000:])
