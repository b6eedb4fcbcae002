/*
 * mw.h -- C ABI of libmwcg: Conjugate Gradient for sparse SPD systems in
 * FP64, double-word (DW), quasi double-word (QDW), triple-word (TW) and
 * quasi triple-word (QTW) arithmetic, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Mukunoki & Ozaki, "Sparse Iterative Solvers Using High-Precision
 * Arithmetic with Quasi Multi-Word Algorithms" (arXiv 2510.13536).
 *   - Problem (Sec. I, Alg. 1, Sec. IV-C): solve A x = b for SPD A, with A
 *     and b in FP64 and x, every CG vector and every CG scalar held in the
 *     chosen arithmetic; the relative-residual test is done in FP64.
 *   - Arithmetic (Sec. III, Alg. 2-10): error-free transformations and the
 *     multi-word add/mul/normalise algorithms; FP64 x multi-word products
 *     drop the terms of the FP64 operand's (zero) lower words.
 *   - Kernels (Sec. IV-B): CSR SpMV with an FP64 matrix and multi-word
 *     vectors, DOT, AXPY.
 *   - Quasi normalisation (Sec. IV-D): QDW/QTW normalise r after its AXPY.
 *
 * Conventions shared by every entry point
 *   Memory:   every pointer argument is a DEVICE pointer unless stated
 *             otherwise; the caller allocates and owns all of it (inputs,
 *             outputs, workspaces).  The library allocates no device memory.
 *   Vectors:  a k-word vector of length n is stored as k "word planes":
 *             k consecutive arrays of n doubles, plane 0 the leading word
 *             (element i of plane w at offset w*n + i).  k = mw_words(a).
 *   Scalars:  a k-word scalar is k consecutive doubles in device memory.
 *   CSR:      row_ptr[n+1] (row_ptr[0] = 0, nondecreasing, row_ptr[n] =
 *             nnz), col_idx[nnz] in [0, n) and ascending within each row,
 *             val[nnz] FP64; all int32.  Symmetric matrices are stored in
 *             full (both triangles).
 *   Streams:  `stream` is a hipStream_t (NULL = the default stream).  All
 *             work is enqueued on it.  mw_spmv, mw_dot, mw_axpy and
 *             mw_elementwise are asynchronous; the solvers return after
 *             synchronising the stream because they must observe
 *             convergence.
 *   Errors:   functions return MW_OK (0), a positive solver status, or a
 *             negative error: MW_EINVAL for a rejected argument (nothing is
 *             enqueued) and MW_EHIP for a HIP runtime error (text available
 *             from mw_last_error()).
 *   Threads:  calls are re-entrant across streams when their workspaces
 *             and outputs are distinct.
 */
#ifndef MW_H
#define MW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The five arithmetics (Sec. I list; Sec. V-B naming CG-FP64 ... CG-QTW). */
typedef enum {
    MW_FP64 = 0,
    MW_DW = 1,
    MW_QDW = 2,
    MW_TW = 3,
    MW_QTW = 4
} mw_arith_t;

/* Return codes. */
enum {
    MW_OK = 0,             /* success / converged                        */
    MW_NOT_CONVERGED = 1,  /* maxit reached; x holds the last iterate    */
    MW_BREAKDOWN = 2,      /* p^T A p <= 0 or a non-finite scalar        */
    MW_EINVAL = -1,        /* invalid argument; nothing enqueued         */
    MW_EHIP = -2           /* HIP runtime error                          */
};

/* Element-wise operation codes for mw_elementwise. */
enum {
    MW_OP_ADD = 0,    /* w = u + v              (Alg. 5 / 7 and quasi forms) */
    MW_OP_MUL = 1,    /* w = u * v              (Alg. 6 / 8 and quasi forms) */
    MW_OP_DXMUL = 2,  /* w = u * v, u FP64      (Alg. 10 rule)              */
    MW_OP_DIV = 3,    /* w = u / v              (long division, see below)  */
    MW_OP_NORM = 4,   /* w = normalise(u)       (QuickTwoSum / VecSum3 Alg. 9) */
    MW_OP_NEG = 5,    /* w = -u                                            */
    MW_OP_TOFP64 = 6  /* w (one plane) = u rounded to FP64                 */
};

/* FP64 CSR matrix; all three arrays in device memory. */
typedef struct {
    int32_t n;              /* rows = columns, >= 1 */
    int32_t nnz;            /* = row_ptr[n], >= 0   */
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} mw_csr_t;

/* Result of a solve (host memory). */
typedef struct {
    int32_t iters;    /* CG iterations performed (SpMVs inside the loop)   */
    int32_t status;   /* MW_OK, MW_NOT_CONVERGED or MW_BREAKDOWN           */
    double rel_res;   /* sqrt(fp64(r^T r)) / ||b||_2 at the last test      */
    double seconds;   /* device time of the solve (HIP events)             */
} mw_cg_info_t;

/* Solver options (host memory); pass NULL for the defaults. */
typedef struct {
    int32_t normalize;  /* QDW/QTW: 1 (default) normalises r after its
                           update once per iteration (Sec. IV-D); 0 skips
                           it (the "-NN" variants of Sec. V-B).  Ignored by
                           the other arithmetics.                            */
    int32_t chunk;      /* iterations launched between two host checks of
                           convergence; 0 = library default               */
    double *history;    /* optional DEVICE array of maxit doubles: entry i
                           receives the relative residual after iteration
                           i+1.  NULL = not recorded.                      */
} mw_cg_opts_t;

/* Number of FP64 words of an arithmetic: 1, 2, 2, 3, 3; -1 if unknown. */
int mw_words(mw_arith_t a);

/* Static text for a return code. */
const char *mw_status_string(int code);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *mw_last_error(void);

/*
 * Element-wise arithmetic over word planes (exposes the Sec. III algorithms
 * for bit-exact testing).  u: k planes of n (one FP64 plane for
 * MW_OP_DXMUL); v: k planes of n (read by ADD, MUL, DXMUL, DIV; may be NULL
 * otherwise); w: k planes of n (one plane for MW_OP_TOFP64).  w may alias u
 * or v.  TW operations are the QTW operation followed by a renormalisation
 * (VecSum then VecSumErrBranch of Fabiano, Muller and Picot, m = 3), the
 * reading taken because the paper cites but does not print the TW
 * algorithms (Sec. III).  Division is long division with FP64 quotient
 * digits: q1 = fl(a1/b1), remainder a - q1*b in the arithmetic, normalised,
 * next digit from its leading word (three digits for 3-word types), result
 * normalised.  Asynchronous.
 */
int mw_elementwise(mw_arith_t a, int op, int32_t n, const double *u, const double *v,
                   double *w, void *stream);

/*
 * y = y + alpha * x (AXPY, Sec. IV-B; Alg. 1 lines 7-8).  alpha: one k-word
 * scalar in device memory; x, y: k planes of n.  FP64: y = fma(alpha, x, y);
 * otherwise y = add(y, mul(alpha, x)).  Bit-identical to the definition.
 * Asynchronous.
 */
int mw_axpy(mw_arith_t a, int32_t n, const double *alpha, const double *x, double *y,
            void *stream);

/* Bytes of device workspace mw_dot needs for length n (256-byte aligned). */
size_t mw_dot_workspace_bytes(mw_arith_t a, int32_t n);

/*
 * result = x^T y (DOT, Sec. IV-B; Alg. 1 lines 6 and 9).  x, y: k planes of
 * n; result: one k-word scalar in device memory.  Products mul(x_i, y_i)
 * are summed with the arithmetic's add in a fixed, run-to-run reproducible
 * order: sequentially over a few elements per thread, then pairwise trees
 * across the wavefront, the workgroup and the workgroup partials.  This
 * order differs from a sequential sum, so the result is not bit-identical
 * to one; its error is a small multiple of the format's unit round-off
 * times sum_i |x_i y_i|.  n = 0 gives 0.  workspace: at least
 * mw_dot_workspace_bytes(a, n) bytes.  Asynchronous.
 */
int mw_dot(mw_arith_t a, int32_t n, const double *x, const double *y, double *result,
           void *workspace, void *stream);

/*
 * y = A x (CSR SpMV, Sec. IV-B; Alg. 1 line 5).  A: FP64 CSR; x, y: k planes
 * of A->n (must not alias).  Each row is accumulated from zero in CSR order,
 * acc = add(acc, a_ij * x_j) with an FP64 x multi-word product (FP64:
 * acc = fma(a_ij, x_j, acc)), so every row is bit-identical to that
 * sequential definition.  No workspace.  Asynchronous.
 */
int mw_spmv(mw_arith_t a, const mw_csr_t *A, const double *x, double *y, void *stream);

/* Bytes of device workspace mw_cg_solve needs (256-byte aligned). */
size_t mw_cg_workspace_bytes(mw_arith_t a, int32_t n, int32_t nnz);

/*
 * CG (Alg. 1 with Sec. IV-C and IV-D).  Solves A x = b from the initial x:
 *   r = b - A x;  p = r;  rho = r^T r;  ||b|| = sqrt(fp64(b^T b));
 *   rho = 0: return at once (0 iterations, MW_OK); maxit = 0: return
 *   MW_NOT_CONVERGED with 0 iterations.
 *   each iteration: q = A p;  sigma = p^T q (sigma <= 0 or non-finite:
 *   MW_BREAKDOWN, x unchanged by that iteration);  alpha = rho / sigma;
 *   x = x + alpha p;  r = r - alpha q;  QDW/QTW: r = normalise(r);
 *   rho' = r^T r;  stop when sqrt(fp64(rho')) / ||b|| < tol (MW_OK) or
 *   after maxit iterations (MW_NOT_CONVERGED);  beta = rho' / rho;
 *   p = r + beta p.
 * A: FP64 CSR, SPD; b: FP64[n]; x: k planes of n, in/out (pass zeros for
 * the paper's x0 = 0); tol >= 0; maxit >= 0; opts may be NULL; workspace:
 * at least mw_cg_workspace_bytes(a, n, nnz) bytes of device memory; info
 * (host) receives iterations, status, final relative residual and time.
 * Returns the status (>= 0) or a negative error.  Synchronises `stream`.
 */
int mw_cg_solve(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, double tol,
                int32_t maxit, const mw_cg_opts_t *opts, void *workspace, mw_cg_info_t *info,
                void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MW_H */
