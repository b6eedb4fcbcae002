// mw_blas.hpp -- internal interface between the BLAS/SpMV and CG parts of
// libmwcg.
#pragma once

#include "mw_common.hpp"

namespace mwk {

// Device-resident state of one CG solve.  Values an iteration produces are
// kept per iteration parity (index i & 1 for iteration i, parity 0 holding
// the initial values): iteration i reads only the other parity's entries,
// which the previous iteration wrote before a kernel boundary, so no
// workgroup ever reads an entry another workgroup of the same kernel
// writes.
struct CgState {
    double rho[2][3];    // r^T r after the iteration of each parity
    double alpha[2][3];  // alpha of the iteration of each parity
    double nb;           // ||b||_2
    double tol;
    double rel_res;      // relative residual at the stop (or the last test)
    double *history;     // optional per-iteration relative residuals
    int32_t run[2];      // the iteration of this parity left the solve running
    int32_t iters[2];    // iteration count after the iteration of this parity
    int32_t brk[2];      // the alpha step of this parity broke down
    int32_t maxit;
    int32_t normalize;
    int32_t stopped;     // set once, when the solve stops (polled by the host)
    int32_t status;      // final status (valid once stopped)
    int32_t iters_final; // final iteration count (valid once stopped)
    int32_t pad;
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
// partials of p^T q go to `slots` (their count to *nslots); the launch does
// nothing but pass the stop on (*run_cur = 0) when *run_prev is 0.
template <int A>
int spmv_launch(const mw_csr_t *M, const mw_spmv_plan_t *plan, const double *x, double *y, double *slots,
                const int32_t *run_prev, int32_t *run_cur, int mode, hipStream_t s, int *nslots = nullptr);

// Number of slots a CG-mode SpMV launch writes (see spmv_launch).
int spmv_slots(const mw_csr_t *M, const mw_spmv_plan_t *plan);

}  // namespace mwh
