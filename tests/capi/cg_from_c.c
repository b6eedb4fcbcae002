/* A caller of libmwcg.so from plain C: no PyTorch, only the header and the
 * HIP runtime's C API for device memory.  2D Poisson (5-point) on a 64 x 64
 * grid with an integer solution x*_i = 1 + (i mod 5) and b = A x*, so the
 * SpMV, dot and AXPY results below are exact integers; then QTW CG from
 * x0 = 0 to 1e-12, and two argument errors.  Prints one line and exits 0
 * when every check holds. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mw.h"

#define NX 64
#define N (NX * NX)

static int fail(const char *what, int rc)
{
    fprintf(stderr, "capi FAIL: %s (rc %d: %s; %s)\n", what, rc, mw_status_string(rc), mw_last_error());
    return 1;
}

#define HIPCHK(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "capi FAIL: %s: %s\n", #call, hipGetErrorString(e_)); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(void)
{
    /* the matrix, columns ascending in every row */
    static int32_t rp[N + 1], ci[5 * N];
    static double va[5 * N], xs[N], b[N], h[3 * N];
    int nnz = 0;
    for (int i = 0; i < N; ++i) {
        const int gx = i % NX, gy = i / NX;
        rp[i] = nnz;
        if (gy > 0) { ci[nnz] = i - NX; va[nnz++] = -1.0; }
        if (gx > 0) { ci[nnz] = i - 1; va[nnz++] = -1.0; }
        ci[nnz] = i; va[nnz++] = 4.0;
        if (gx < NX - 1) { ci[nnz] = i + 1; va[nnz++] = -1.0; }
        if (gy < NX - 1) { ci[nnz] = i + NX; va[nnz++] = -1.0; }
    }
    rp[N] = nnz;
    double xx = 0.0;
    for (int i = 0; i < N; ++i) {
        xs[i] = 1.0 + (double)(i % 5);
        xx += xs[i] * xs[i];
    }
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int z = rp[i]; z < rp[i + 1]; ++z) s += va[z] * xs[ci[z]];
        b[i] = s;
    }

    int32_t *d_rp, *d_ci;
    double *d_va, *d_b, *d_x, *d_y, *d_xs3, *d_dot, *d_alpha;
    void *d_ws, *d_dws;
    HIPCHK(hipMalloc((void **)&d_rp, sizeof(rp)));
    HIPCHK(hipMalloc((void **)&d_ci, sizeof(int32_t) * nnz));
    HIPCHK(hipMalloc((void **)&d_va, sizeof(double) * nnz));
    HIPCHK(hipMalloc((void **)&d_b, sizeof(b)));
    HIPCHK(hipMalloc((void **)&d_y, sizeof(b)));
    HIPCHK(hipMalloc((void **)&d_x, 3 * sizeof(b)));
    HIPCHK(hipMalloc((void **)&d_xs3, 3 * sizeof(b)));
    HIPCHK(hipMalloc((void **)&d_dot, 3 * sizeof(double)));
    HIPCHK(hipMalloc((void **)&d_alpha, sizeof(double)));
    HIPCHK(hipMemcpy(d_rp, rp, sizeof(rp), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_ci, ci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_va, va, sizeof(double) * nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_b, b, sizeof(b), hipMemcpyHostToDevice));
    const mw_csr_t A = {N, nnz, d_rp, d_ci, d_va};

    /* FP64 SpMV: y = A x* = b exactly */
    HIPCHK(hipMemcpy(d_x, xs, sizeof(xs), hipMemcpyHostToDevice));
    int rc = mw_spmv(MW_FP64, &A, d_x, d_y, NULL);
    if (rc != MW_OK) return fail("mw_spmv", rc);
    HIPCHK(hipMemcpy(h, d_y, sizeof(b), hipMemcpyDeviceToHost));
    if (memcmp(h, b, sizeof(b)) != 0) return fail("mw_spmv result", 0);

    /* FP64 AXPY: y = y + 2 x* */
    const double two = 2.0;
    HIPCHK(hipMemcpy(d_alpha, &two, sizeof(double), hipMemcpyHostToDevice));
    rc = mw_axpy(MW_FP64, N, d_alpha, d_x, d_y, NULL);
    if (rc != MW_OK) return fail("mw_axpy", rc);
    HIPCHK(hipMemcpy(h, d_y, sizeof(b), hipMemcpyDeviceToHost));
    for (int i = 0; i < N; ++i)
        if (h[i] != b[i] + 2.0 * xs[i]) return fail("mw_axpy result", 0);

    /* QTW dot of x* (word planes x*, 0, 0) with itself: the exact integer */
    HIPCHK(hipMemset(d_xs3, 0, 3 * sizeof(b)));
    HIPCHK(hipMemcpy(d_xs3, xs, sizeof(xs), hipMemcpyHostToDevice));
    const size_t dws = mw_dot_workspace_bytes(MW_QTW, N);
    HIPCHK(hipMalloc(&d_dws, dws));
    rc = mw_dot(MW_QTW, N, d_xs3, d_xs3, d_dot, d_dws, NULL);
    if (rc != MW_OK) return fail("mw_dot", rc);
    double dot[3];
    HIPCHK(hipMemcpy(dot, d_dot, sizeof(dot), hipMemcpyDeviceToHost));
    if (dot[0] != xx || dot[1] != 0.0 || dot[2] != 0.0) return fail("mw_dot result", 0);

    /* QTW CG from x0 = 0 */
    const size_t wsb = mw_cg_workspace_bytes(MW_QTW, N, nnz);
    HIPCHK(hipMalloc(&d_ws, wsb));
    HIPCHK(hipMemset(d_x, 0, 3 * sizeof(b)));
    mw_cg_info_t info;
    rc = mw_cg_solve(MW_QTW, &A, d_b, d_x, 1e-12, 10 * N, NULL, d_ws, &info, NULL);
    if (rc != MW_OK || info.status != MW_OK) return fail("mw_cg_solve", rc);
    HIPCHK(hipMemcpy(h, d_x, 3 * sizeof(b), hipMemcpyDeviceToHost));
    double err = 0.0;
    for (int i = 0; i < N; ++i) err = fmax(err, fabs(h[i] - xs[i]));
    if (!(err < 1e-9) || info.iters <= 0 || !(info.rel_res < 1e-12)) return fail("mw_cg_solve result", 0);

    /* argument errors: nothing enqueued, MW_EINVAL */
    if (mw_cg_solve(MW_QTW, &A, d_b, d_x, 1e-12, -1, NULL, d_ws, &info, NULL) != MW_EINVAL)
        return fail("maxit < 0 accepted", 0);
    if (mw_dot(MW_QTW, N, d_xs3, d_xs3, d_dot, NULL, NULL) != MW_EINVAL) return fail("NULL workspace accepted", 0);

    printf("capi ok: QTW CG %d iterations, rel. residual %.3e, max |x - x*| %.3e\n", info.iters, info.rel_res, err);
    hipFree(d_rp); hipFree(d_ci); hipFree(d_va); hipFree(d_b); hipFree(d_y); hipFree(d_x); hipFree(d_xs3);
    hipFree(d_dot); hipFree(d_alpha); hipFree(d_ws); hipFree(d_dws);
    return 0;
}
