// mw_blas.hpp -- internal interface between the BLAS/SpMV and CG parts of
// libmwcg.
#pragma once

#include "mw_common.hpp"

namespace mwk {

// Device-resident state of one CG solve.
struct CgState {
    double rho[3];    // r^T r of the current iterate
    double alpha[3];
    double beta[3];
    double nb;        // ||b||_2
    double tol;
    double rel_res;   // last relative residual
    double *history;  // optional per-iteration relative residuals
    int32_t active;   // 1 while iterating
    int32_t status;   // MW_OK / MW_NOT_CONVERGED / MW_BREAKDOWN
    int32_t iters;
    int32_t maxit;
    int32_t normalize;
    int32_t x_due;    // the stopping iteration's x update is still to be applied
    int32_t pad[2];
};

}  // namespace mwk

namespace mwh {

// Bytes of a SpMV plan buffer for an n x n matrix with nnz entries.
size_t plan_bytes(int32_t n, int32_t nnz);

// Builds a plan (SELL-64, or the CSR fallback) in `buffer`; synchronises s.
int plan_build(const mw_csr_t *A, void *buffer, size_t bytes, mw_spmv_plan_t *plan, hipStream_t s);

// Most reduction slots any CG-mode SpMV launch writes for n rows.
int spmv_max_slots(int32_t n);

// y = A x.  plan == nullptr or plan->format == MW_FMT_CSR: CSR kernel on M;
// else the SELL-64 kernel.  mode 1 (CG): x is p, y is q, the workgroup
// partials of p^T q go to `slots` (their count to *nslots) and the launch
// is skipped on the device once st->active is 0.
template <int A>
int spmv_launch(const mw_csr_t *M, const mw_spmv_plan_t *plan, const double *x, double *y, double *slots,
                const mwk::CgState *st, int mode, hipStream_t s, int *nslots = nullptr);

}  // namespace mwh
