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
// Loads of the matrix stream in the planned SpMV.  For 3-word vectors the
// CG working set (four vectors of 24 bytes per row) competes with the
// matrix stream for the 256 MB Infinity Cache; the matrix entries are used
// once per SpMV, so they are loaded non-temporally there.  For 1- and
// 2-word vectors plain loads measured faster.
template <int A, typename T>
__device__ __forceinline__ T load_matrix(const T *p)
{
    if constexpr (words(A) == 3) return __builtin_nontemporal_load(p);
    else return *p;
}

// Sum of one row of a SELL-64 slice: entries z0, z0 + 64, ... < z1 (the
// lane's column of the slice), in order, from zero; padding (col < 0) is
// skipped.  Two entries are loaded ahead of their dependent adds.
template <int A>
__device__ __forceinline__ Num<A> sell_row_sum(int z0, int z1, const int32_t *__restrict__ sc,
                                               const double *__restrict__ sv, const double *__restrict__ x, long n)
{
    Num<A> acc = zero<A>();
    int z = z0;
    for (; z + 64 < z1; z += 128) {
        const double a0 = load_matrix<A>(sv + z), a1 = load_matrix<A>(sv + z + 64);
        const int c0 = load_matrix<A>(sc + z), c1 = load_matrix<A>(sc + z + 64);
        const Num<A> x0 = load<A>(x, n, c0 < 0 ? 0 : c0);
        const Num<A> x1 = load<A>(x, n, c1 < 0 ? 0 : c1);
        if (c0 >= 0) acc = row_step<A>(acc, a0, x0);
        if (c1 >= 0) acc = row_step<A>(acc, a1, x1);
    }
    if (z < z1) {
        const double a0 = load_matrix<A>(sv + z);
        const int c0 = load_matrix<A>(sc + z);
        const Num<A> x0 = load<A>(x, n, c0 < 0 ? 0 : c0);
        if (c0 >= 0) acc = row_step<A>(acc, a0, x0);
    }
    return acc;
}

// Sum over the 64 lanes of a wavefront (shuffle tree, offsets 32 .. 1);
// valid in lane 0.
template <int A>
__device__ __forceinline__ Num<A> wave_sum(Num<A> v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = add<A>(v, shfl_down<A>(v, off));
    return v;
}

}  // namespace mwk

namespace mwh {

// Exclusive scan of 64 * width[0..ns) into slice_ptr[0..ns], 64-bit total
// into *total (one workgroup).
int launch_sell_scan(int ns, const int32_t *width, int32_t *slice_ptr, long long *total, hipStream_t s);


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
