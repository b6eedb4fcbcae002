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
 *   Scalars:  a scalar is mw_scalar_words(a) consecutive doubles in device
 *             memory (= k, except for the mixed types, whose scalars are
 *             multi-word while their vectors are FP64).
 *   CSR:      row_ptr[n+1] (row_ptr[0] = 0, nondecreasing, row_ptr[n] =
 *             nnz), col_idx[nnz] in [0, n) and ascending within each row,
 *             val[nnz] FP64; all int32.  Symmetric matrices are stored in
 *             full (both triangles).
 *   Sizes:    n (rows, vector length) and nnz at most MW_MAX_N = 2^31 -
 *             2^16, so that no 32-bit index a kernel forms past the end of
 *             its range (a partial tile, a row group, a padded slice)
 *             overflows; larger sizes are MW_EINVAL (byte-count queries
 *             return 0).
 *   Streams:  `stream` is a hipStream_t (NULL = the default stream).  All
 *             work is enqueued on it.  mw_spmv, mw_dot, mw_axpy and
 *             mw_elementwise are asynchronous; the solvers return after
 *             synchronising the stream because they must observe
 *             convergence.
 *   Errors:   functions return MW_OK (0), a positive solver status, or a
 *             negative error: MW_EINVAL for a rejected argument (nothing is
 *             enqueued) and MW_EHIP for a HIP runtime error (details from
 *             mw_last_error()).
 *   Threads:  calls are re-entrant across streams when their workspaces
 *             and outputs are distinct.  The solvers' own streams, captured
 *             graphs and pinned host flags are kept per calling thread (the
 *             streams also per device, the one current at the call), and
 *             held until the process ends.
 */
#ifndef MW_H
#define MW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest n and nnz (see Sizes above). */
#define MW_MAX_N 2147418112

/* The five arithmetics (Sec. I list; Sec. V-B naming CG-FP64 ... CG-QTW),
 * and QTWE: QTW with VecSum3 (Alg. 9) after every operation, the
 * every-operation end of the normalisation placement Sec. IV-D and VI leave
 * open (3 words; r gets no extra normalisation; the QDW counterpart of this
 * placement is DW itself).  The quadruple-word formats the paper names in
 * Sec. I without giving their algorithms: QW (4 words; the quad-double
 * algorithms of Hida, Li and Bailey) and QQW (4 words; read as Alg. 7, 8,
 * 10 carried one order further, with VecSum4 normalising r in CG like the
 * other quasi types).  Mixed precision (future work in Sec. VI): MW_MXDW and
 * MW_MXQTW keep every vector in FP64 (one plane) and accumulate SpMV rows
 * (each rounded once to FP64) and dots (kept multi-word) in DW / QTW;
 * alpha and beta are DW / QTW quotients rounded to FP64 for FP64 fma
 * updates.  Their scalars (dot results, alpha arguments) have
 * mw_scalar_words() words; mw_elementwise and mw_csr_grad reject them (their
 * vectors are FP64: use MW_FP64 there).  With Jacobi preconditioning their
 * z = D r is an FP64 vector too (z_i = fl(d_i r_i)). */
typedef enum {
    MW_FP64 = 0,
    MW_DW = 1,
    MW_QDW = 2,
    MW_TW = 3,
    MW_QTW = 4,
    MW_QTWE = 5,
    MW_QW = 6,
    MW_QQW = 7,
    MW_MXDW = 8,
    MW_MXQTW = 9
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

/* Storage formats of a SpMV plan. */
enum {
    MW_FMT_CSR = 0,     /* the caller's CSR arrays are used as given        */
    MW_FMT_SELL64 = 1,  /* sliced ELLPACK, 64-row slices (see mw_spmv_plan) */
    MW_FMT_CSRVEC = 2   /* the CSR arrays, several lanes per row
                           (see mw_spmv_plan_rows)                          */
};

/* A SpMV plan (host struct; the arrays it points to live in the caller's
 * plan buffer in device memory, plus the caller's CSR arrays).  SELL64
 * storage is counted in 64-entry slots: slice s owns slots
 * slice_ptr[s] / 64 .. slice_ptr[s + 1] / 64 - 1, one per entry of its
 * longest row. */
typedef struct {
    int32_t n, nnz;
    int32_t format;             /* MW_FMT_SELL64 (or MW_FMT_CSR as fallback)
                                   from mw_spmv_plan; MW_FMT_CSRVEC from
                                   mw_spmv_plan_rows                          */
    int32_t nslices;            /* ceil(n / 64)                               */
    int64_t stored;             /* SELL64: entries stored, padding included    */
    const int32_t *slice_ptr;   /* SELL64: nslices + 1 offsets (entries)      */
    const int32_t *col;         /* SELL64: column of each entry of an explicit-
                                   column slice, -1 = padding (unused entries
                                   of diagonal-slot slices are unspecified)   */
    const double *val;          /* SELL64: value of each entry (0 = padding)   */
    const int32_t *slot_off;    /* SELL64: per slot of a diagonal-slot slice,
                                   the column offset (column - row) it holds  */
    const uint64_t *slot_mask;  /* SELL64: per slot, bit l set when row
                                   64 s + l has an entry in that slot; 0 for
                                   every slot of an explicit-column slice     */
    int32_t ndiag;              /* SELL64: slices stored as diagonal slots    */
    int32_t lanes;              /* CSRVEC: lanes per row (2, 4, ..., 64)      */
    mw_csr_t csr;               /* the source matrix                          */
} mw_spmv_plan_t;

/* Result of a solve (host memory). */
typedef struct {
    int32_t iters;    /* CG iterations performed (SpMVs inside the loop)   */
    int32_t status;   /* MW_OK, MW_NOT_CONVERGED or MW_BREAKDOWN           */
    double rel_res;   /* sqrt(fp64(r^T r)) / ||b||_2 at the last test      */
    double seconds;   /* device time of the solve (HIP events)             */
} mw_cg_info_t;

/* Optional per-kernel timing of a solve (host memory).  When given, the
 * solver brackets every kernel launch of the iteration loop with HIP events
 * on `stream` and adds, over the iterations that ran to completion, the
 * device time (ms) and the number of launches of each kernel class.
 * Only the classes selected by `mask` are timed (each timed launch adds an
 * event pair); a timed solve launches its kernels directly instead of
 * replaying a captured graph.  Leave the pointer NULL otherwise. */
enum {
    MW_PROF_SPMV = 0,      /* q = A p and the p^T q partials               */
    MW_PROF_UPDATE_R = 1,  /* x, r updates, normalisation, r^T r partials  */
    MW_PROF_UPDATE_P = 2,  /* p = r + beta p                               */
    MW_PROF_FINAL = 3,     /* scalar finalisers (alpha, beta, test)        */
    MW_PROF_CLASSES = 4
};
typedef struct {
    double ms[MW_PROF_CLASSES];          /* out: summed device time          */
    int64_t launches[MW_PROF_CLASSES];   /* out: launches timed              */
    int32_t mask;                        /* in: bit c times class c; 0 = all */
    int32_t reserved;
} mw_cg_prof_t;

/* Launch shape of the solvers' kernels (a set-up choice, not part of the
 * paper's method; results of a solve depend on it only through the order
 * in which per-workgroup dot partials are combined).  A field <= 0 means
 * "not set". */
typedef struct {
    int32_t spmv_grid;       /* workgroups of the SpMV (batched: of every
                                slice kernel), 8 .. 2048                    */
    int32_t update_grid;     /* single system: workgroups of the two
                                vector-update kernels, 8 .. 2048            */
    int32_t update_threads;  /* single system: threads per update
                                workgroup, 256, 512 or 1024                 */
    int32_t chunk;           /* iterations per captured chunk, 1 .. 4096   */
    int32_t lanes;           /* lanes per row, 2, 4, ..., 64: single system,
                                of the vector-row plan the solver builds
                                itself (MW_FMT_CSRVEC); batched, of its
                                vector-row slices                          */
    double us_per_iteration; /* set by the tuners: measured device time per
                                iteration of the chosen shape              */
} mw_shape_t;

/* Preconditioners of mw_cg_solve (opts->precond). */
enum {
    MW_PRECOND_NONE = 0,    /* plain CG, Alg. 1                              */
    MW_PRECOND_JACOBI = 1   /* M^-1 = diag(fl(1 / a_ii)), an extension: the
                               paper names preconditioning as future work
                               (Sec. VI)                                     */
};

/* Solver options (host memory); pass NULL for the defaults. */
typedef struct {
    int32_t normalize;  /* QDW/QTW: K >= 1 normalises r right after its
                           update in iterations K, 2K, ... -- 1 (default)
                           is every iteration (Sec. IV-D), other K explore
                           the frequency Sec. VI leaves open; 0 never (the
                           "-NN" variants of Sec. V-B).  Ignored by the
                           other arithmetics; < 0: MW_EINVAL.              */
    int32_t chunk;      /* iterations launched between two host checks of
                           convergence; 0 = library default.  The single
                           solver rounds it up to an even number.         */
    double *history;    /* optional DEVICE array of maxit doubles: entry i
                           receives the relative residual after iteration
                           i+1.  NULL = not recorded.                      */
    mw_cg_prof_t *prof; /* optional HOST struct for per-kernel timing      */
    const mw_spmv_plan_t *plan;  /* optional plan of A (mw_spmv_plan or
                           mw_spmv_plan_rows).  NULL: the solver builds one
                           -- vector rows (MW_FMT_CSRVEC) when n <= 2^18 and
                           rows average 32 or more entries, or when SELL64
                           would pad too much (the CSR fallback) and rows
                           average 16 or more; else SELL64 inside the
                           workspace.  Its lanes per row: shape->lanes,
                           else a tuned shape's, else about 8 entries per
                           lane in MW_FP64 and 16 in the other arithmetics.
                           A plan of another matrix, or whose fields do not
                           fit its format (see mw_spmv_planned): MW_EINVAL */
    int32_t no_graph;   /* nonzero: launch each kernel directly instead of
                           replaying a captured hipGraph of a chunk       */
    int32_t precond;    /* MW_PRECOND_NONE (0): Alg. 1.  MW_PRECOND_JACOBI:
                           Jacobi-preconditioned CG (see mw_cg_solve), for
                           the single and the batched solver              */
    const mw_shape_t *shape;  /* optional launch shape; its set fields take
                           precedence over a tuned shape (mw_cg_tune), which
                           takes precedence over the MW_SGRID / MW_UGRID /
                           MW_UNT environment overrides and the built-in
                           shape.  chunk above takes precedence over
                           shape->chunk.  Invalid values: MW_EINVAL.       */
    int32_t normalize_p;  /* 0 (default): only r is normalised (Sec. IV-D).
                           1: in the iterations that normalise r, p is
                           normalised too, as it enters p = r + beta p (a
                           placement variant for the frequency question of
                           Sec. VI: with it every normalize = K converges
                           where r alone breaks down).  Plain CG of the
                           single solver only; other values, or with a
                           preconditioner or the batched solver:
                           MW_EINVAL.                                      */
} mw_cg_opts_t;

/* Number of FP64 words (planes) of a vector element of an arithmetic:
 * 1, 2, 2, 3, 3, 3, 4, 4 and 1 for the mixed types; -1 if unknown. */
int mw_words(mw_arith_t a);

/* Words of a scalar of arithmetic a (a dot result, an axpy alpha): mw_words
 * for all but the mixed types (MW_MXDW: 2, MW_MXQTW: 3); < 0 if invalid. */
int mw_scalar_words(mw_arith_t a);

/* Static text for a return code. */
const char *mw_status_string(int code);

/* Details of the last failed call on this thread: the HIP error of an
 * MW_EHIP, or the cause of an MW_EINVAL that is more than a rejected
 * argument (a failed CSR check, batched padding beyond the workspace, a
 * tuner run that stopped early); "" otherwise.  Every status-returning
 * call clears it on entry. */
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
 * y = y + alpha * x (AXPY, Sec. IV-B; the x and r updates of Alg. 1).  alpha: one
 * scalar (mw_scalar_words(a) words) in device memory; x, y: k planes of n.
 * FP64: y = fma(alpha, x, y); mixed types: y = fma(fp64(alpha), x, y);
 * otherwise y = add(y, mul(alpha, x)).  Bit-identical to the definition.
 * Asynchronous.
 */
int mw_axpy(mw_arith_t a, int32_t n, const double *alpha, const double *x, double *y,
            void *stream);

/* Bytes of device workspace mw_dot needs for length n (256-byte aligned). */
size_t mw_dot_workspace_bytes(mw_arith_t a, int32_t n);

/*
 * result = x^T y (DOT, Sec. IV-B; p^T q and r^T r in Alg. 1).  x, y: k planes of
 * n; result: one scalar (mw_scalar_words(a) words) in device memory; the
 * mixed types sum the exact products of their FP64 entries in DW / QTW.
 * Products mul(x_i, y_i)
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

/* Largest n mw_dot_noalloc accepts (2^25 elements). */
#define MW_DOT_NOALLOC_MAX_N 33554432

/*
 * mw_dot without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and summation
 * order as mw_dot, so the result is bit-identical to mw_dot's.  The
 * per-workgroup partial sums live in a static device array of the library
 * (512 KiB per GPU, held until the process ends); the library allocates
 * nothing.  n in [0, MW_DOT_NOALLOC_MAX_N]; a larger n returns MW_EINVAL
 * (mw_last_error says why).  Calls that overlap on one GPU (several
 * streams, threads or processes' graphs at once) share that array and race:
 * serialise them.  The first call on a device looks up the array's address
 * there (a host-side query, no allocation).  Asynchronous.
 */
int mw_dot_noalloc(mw_arith_t a, int32_t n, const double *x, const double *y, double *result,
                   void *stream);

/*
 * y = A x (CSR SpMV, Sec. IV-B; q = A p in Alg. 1).  A: FP64 CSR; x, y: k planes
 * of A->n (must not alias).  Each row is accumulated from zero in CSR order,
 * acc = add(acc, a_ij * x_j) with an FP64 x multi-word product (FP64:
 * acc = fma(a_ij, x_j, acc)), so every row is bit-identical to that
 * sequential definition; the mixed types accumulate in DW / QTW and round
 * each row once to FP64.  No workspace.  Asynchronous.
 */
int mw_spmv(mw_arith_t a, const mw_csr_t *A, const double *x, double *y, void *stream);

/*
 * Checks a CSR matrix on the device (a set-up step, not part of the
 * paper's method): row_ptr[0] = 0, row_ptr[n] = nnz, row_ptr
 * non-decreasing, every column index in [0, n).  Reads row_ptr[0 .. n] and
 * col_idx[0 .. nnz) only, so it is safe on arrays of those lengths
 * whatever they hold, whereas the other entry points trust these
 * properties and may read out of bounds without them.  Returns MW_OK or
 * MW_EINVAL (mw_last_error names the first failed property).  With
 * MW_CHECK_CSR=1 in the environment (read once per process) every entry
 * point that reads a matrix runs this check first and returns its
 * MW_EINVAL.  Synchronises `stream`.
 */
int mw_csr_check(const mw_csr_t *A, void *stream);


/* Bytes of device memory mw_spmv_plan needs for an n x n matrix with nnz
 * entries (256-byte aligned); 0 for invalid sizes. */
size_t mw_spmv_plan_bytes(int32_t n, int32_t nnz);

/*
 * Re-lays A out for the GPU (a set-up step, not part of the paper's
 * method): slices of 64 consecutive rows, one per wavefront, each lane
 * owning one row; each slice is padded to its longest row, width w.
 * Entries j = 2m and 2m + 1 of row 64 s + l are stored at
 * slice_ptr[s] + 128 m + 2 l (+1), an odd last entry (j = w - 1) at
 * slice_ptr[s] + 128 (w / 2) + l, so every wavefront load is contiguous and
 * each lane reads two entries per 16-byte load.  A slice whose rows can be
 * assigned, each in its own CSR order, to w slots that each hold one
 * column offset (column - row) for all its rows is stored as diagonal
 * slots: values only, plus slot_off / slot_mask per slot (stencil and
 * banded slices); other slices keep explicit columns.  Row contents and
 * their order are kept, so products computed from the plan are
 * bit-identical to those from the CSR arrays.  When the padding would
 * exceed the buffer (rows of very uneven length inside one slice) the plan
 * falls back to format MW_FMT_CSR.  A's arrays must stay valid while the
 * plan is used.  buffer: device memory of at least mw_spmv_plan_bytes
 * bytes; plan: host struct filled on success.  Synchronises `stream`.
 */
int mw_spmv_plan(const mw_csr_t *A, void *buffer, size_t bytes, mw_spmv_plan_t *plan, void *stream);

/*
 * A plan for matrices with few, long rows (a set-up step, not part of the
 * paper's method): the SpMV of a SELL64 plan gives each row one lane, so
 * such a matrix (say 18,000 rows of ~400 entries) leaves most of the GPU
 * idle.  This format keeps A's CSR arrays and gives each row `lanes` lanes
 * (2, 4, ..., 64; 0 chooses about eight entries per lane for the average
 * row): lane t adds the row's entries t, t + lanes, ... in CSR order from
 * zero, and the lanes' sums are combined by a fixed halving tree (lane t
 * adds lane t + d for d = lanes/2, ..., 1).  The result is deterministic but
 * associated differently from mw_spmv's CSR order: within the format's
 * accuracy bound (Sec. III error of a sum of len products, over a path of
 * ceil(len / lanes) + log2(lanes) operations), not bit-identical.  No
 * device memory; A's arrays must stay valid while the plan is used.
 * Returns MW_EINVAL for another `lanes`.  Host only (no stream work).
 */
int mw_spmv_plan_rows(const mw_csr_t *A, int32_t lanes, mw_spmv_plan_t *plan);

/* y = A x with a plan: for MW_FMT_SELL64 and MW_FMT_CSR plans the same
 * result, bit for bit, as mw_spmv; for MW_FMT_CSRVEC plans the row order
 * described at mw_spmv_plan_rows.  A plan whose fields do not fit its
 * format (unknown format, SELL64 arrays missing, lanes not 2, 4, ..., 64,
 * n not its matrix's): MW_EINVAL.  Asynchronous. */
int mw_spmv_planned(mw_arith_t a, const mw_spmv_plan_t *plan, const double *x, double *y, void *stream);

/*
 * Gradient of a loss with respect to the stored entries of A, for
 * x = A^-1 b and lam = A^-T (dL/dx) (the adjoint solve; for SPD A the same
 * CG as the forward solve): grad_val[k] = -(lam_i * x_j) for the k-th
 * stored entry (i, j), the product formed in the arithmetic and rounded to
 * FP64.  dL/db is lam itself.  (The adjoint is a pattern added beside the
 * paper's method; each of its solves is Alg. 1.)  lam, x: k planes of n;
 * grad_val: FP64[nnz], CSR order.  Asynchronous.
 */
int mw_csr_grad(mw_arith_t a, const mw_csr_t *A, const double *lam, const double *x, double *grad_val,
                void *stream);

/* Bytes of device workspace mw_cg_solve needs (256-byte aligned): the
 * vectors r and q, the search direction (3-word types: two buffers, so
 * that x takes the updates of two iterations in one pass), the Jacobi
 * reciprocals, partial sums, the solver state and room for a SpMV plan of
 * A. */
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
 * With opts->precond = MW_PRECOND_JACOBI the textbook preconditioned CG
 * runs instead, with M^-1 the FP64 diagonal d_i = fl(1 / a_ii) applied as
 * the FP64 x multi-word product (FP64 and the mixed types: one rounded
 * product):
 *   r = b - A x;  z = D r;  p = z;  rho = r^T z;  rr = r^T r;  stop at once
 *   when fp64(rr) = 0;  each iteration as above up to the normalisation of
 *   r, then z = D r;  rho' = r^T z;  rr = r^T r;  the test uses
 *   sqrt(fp64(rr)) / ||b|| (the paper's residual test);  beta = rho' / rho;
 *   p = z + beta p.  A row without a nonzero stored diagonal entry makes
 *   d_i infinite: MW_BREAKDOWN at the first test.
 * A: FP64 CSR, SPD; b: FP64[n]; x: k planes of n, in/out (pass zeros for
 * the paper's x0 = 0); tol >= 0; maxit >= 0; opts may be NULL; workspace:
 * at least mw_cg_workspace_bytes(a, n, nnz) bytes of device memory; info
 * (host) receives iterations, status, final relative residual and time.
 * Returns the status (>= 0) or a negative error.  The solve runs on a
 * stream of the library's own, ordered after the work already enqueued on
 * `stream`, and is complete when the call returns.  Iterations are enqueued
 * in chunks (opts->chunk, default 32, rounded up to an even number) as a
 * captured hipGraph that is reused by later calls with the same arguments
 * on the same thread (up to eight captured chunks per thread, the least
 * recently used replaced); every kernel exits at once after the stop, and
 * the host checks the stop flag once per chunk.  The result is run-to-run
 * reproducible.
 */
int mw_cg_solve(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, double tol,
                int32_t maxit, const mw_cg_opts_t *opts, void *workspace, mw_cg_info_t *info,
                void *stream);

/*
 * The SpMV plan mw_cg_solve builds for itself in arithmetic a when
 * opts->plan is NULL (a set-up step, not part of the paper's method; the
 * rule is described at opts->plan): vector rows (MW_FMT_CSRVEC, nothing
 * written to `buffer`), or SELL64 / its CSR fallback in `buffer`, which
 * must then hold mw_spmv_plan_bytes(n, nnz) bytes of device memory (else
 * MW_EINVAL; NULL with bytes = 0 is fine for vector rows).  lanes: 0 = the
 * solver's own (a tuned shape's, else its rule), or 2, 4, ..., 64.  Passed
 * as opts->plan it gives the solver's default results without its per-call
 * set-up.  plan: host struct filled on success.  Synchronises `stream`
 * unless vector rows are taken for the matrix's size.
 */
int mw_cg_plan(mw_arith_t a, const mw_csr_t *A, int32_t lanes, void *buffer, size_t bytes, mw_spmv_plan_t *plan,
               void *stream);

/* Bytes of device workspace mw_cg_solve_batched needs for nsys systems of
 * n rows and nnz entries in total (256-byte aligned). */
size_t mw_cg_batched_workspace_bytes(mw_arith_t a, int32_t nsys, int32_t n, int32_t nnz);

/*
 * Solves nsys independent SPD systems together: the CG of mw_cg_solve
 * (Alg. 1, Sec. IV-C/IV-D) runs for every system with its own scalars,
 * iteration count, FP64 stopping test and status.  A is the block-diagonal
 * matrix of the systems (each row's columns inside its own system's
 * rows); system s owns rows sys_row_off[s] .. sys_row_off[s+1]-1.
 * sys_row_off: HOST array of nsys + 1 nondecreasing offsets, [0] = 0,
 * [nsys] = A->n (empty systems are allowed and finish at once).  b: FP64[n];
 * x: k planes of n, in/out; tol, maxit: as mw_cg_solve, for every system.
 * iters, status: DEVICE int32[nsys] outputs (may be NULL); rel_res: DEVICE
 * double[nsys] output, each system's last relative residual (may be NULL).
 * info (host, may be NULL): iters = the largest count, status = the worst
 * status (MW_OK < MW_NOT_CONVERGED < MW_BREAKDOWN), seconds.  opts:
 * normalize, chunk (default 16), no_graph, shape (spmv_grid, chunk) and
 * precond (Jacobi per system as in mw_cg_solve, each system's d_i from its
 * own rows) are honoured; shape->lanes sets the lanes per row of the
 * vector-row slices (below).  All systems advance in lockstep, five kernels
 * per iteration (six when there are vector-row slices) replayed from a
 * captured hipGraph; a converged system's rows cost a flag test per 64-row
 * slice afterwards.  The matrix is copied into a SELL-64 layout whose
 * slices never straddle two systems, except 64-row slices whose longest row
 * has at least 9 entries and more than 4 times their average: those are
 * summed as vector rows straight from A (L lanes per row, L from the
 * slice's lengths unless shape->lanes is set; the row order of
 * mw_spmv_plan_rows with the same L), so a few very long rows cost no
 * padding.
 * Each system gives the same results whatever the other systems are, but
 * its dots are summed per 64-row slice, so they need not be bit-identical
 * to a single-system mw_cg_solve.  Returns the worst status or a negative
 * error (MW_EINVAL also when the SELL-64 padding of the remaining slices
 * would still exceed the workspace: many slices of rows shorter than 9
 * entries beside much longer ones).
 * Synchronises `stream`.
 */
int mw_cg_solve_batched(mw_arith_t a, int32_t nsys, const int32_t *sys_row_off, const mw_csr_t *A,
                        const double *b, double *x, double tol, int32_t maxit, const mw_cg_opts_t *opts,
                        void *workspace, int32_t *iters, int32_t *status, double *rel_res,
                        mw_cg_info_t *info, void *stream);

/*
 * Launch-shape autotuner (a set-up step, not part of the paper's method).
 * Times `iters` CG iterations (tol = 0, so every candidate runs the same
 * iterations; x is scratch and overwritten, b as for mw_cg_solve, b != 0)
 * for each candidate shape -- SpMV grids 1024, 1280, 1536, 1792, 2048 x
 * update grids 512, 1024, 2048 at 256 threads, and when the solver would
 * build a vector-row plan (see opts->plan), x its lanes per row, half and
 * twice that; candidates that clamp to the same launch counted once -- on
 * `stream`'s device, each timed as the best of three runs after one that
 * captures its graph.  The fastest (the untuned shape unless another is
 * more than 1 % faster) goes to *best and into a per-process table keyed
 * by (a, n, nnz): later mw_cg_solve calls on matrices of that size use it
 * unless opts->shape sets a field.  With MW_TUNE_CACHE=<file> in the
 * environment the table is also kept in that file, one JSON object per
 * line keyed by the device (architecture and compute units) and the size:
 * read at the process's first shape lookup (the current device's lines),
 * rewritten after every tuner result (mw_cg_batched_tune's too) through a
 * temporary file renamed over it; a file that cannot be read or written
 * is skipped.  iters: 2 .. 4096.  workspace: as mw_cg_solve.  Synchronises `stream`.
 * Returns MW_OK or a negative error (MW_EINVAL also when b = 0 or the
 * iterations break down before iters).
 */
int mw_cg_tune(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, int32_t iters, void *workspace,
               mw_shape_t *best, void *stream);

/*
 * The same for mw_cg_solve_batched: candidate slice-kernel grids 256, 512,
 * 1024, 1536, 2048, each timed over `iters` lockstep iterations of all
 * systems (tol = 0), then, when the batch has vector-row slices, lanes per
 * row 2, 4, ..., 64 on the best grid (rows per wavefront 64 / lanes; lanes
 * change how those rows' sums are associated); the table key is (a, n,
 * nnz, nsys).  Arguments as mw_cg_solve_batched plus iters (2 .. 4096) and
 * *best.
 */
int mw_cg_batched_tune(mw_arith_t a, int32_t nsys, const int32_t *sys_row_off, const mw_csr_t *A,
                       const double *b, double *x, int32_t iters, void *workspace, mw_shape_t *best,
                       void *stream);

/*
 * The launch shape a solve of an n x n matrix with nnz entries would use
 * now with opts->shape unset (nsys = 0: mw_cg_solve; nsys >= 1:
 * mw_cg_solve_batched of nsys systems, whose slice grid depends on the
 * systems' slice count, reported here as 0 when not tuned, and lanes the
 * tuned lanes per row of its vector-row slices, 0 for each slice's rule): a tuned shape,
 * else the environment overrides, else the built-in one, with grids
 * clamped to what the matrix needs.  lanes: the lanes per row when a solve
 * would build a vector-row plan by the matrix's size (see opts->plan), else
 * 0 and the grid of SELL64 (a matrix that a solve gives vector rows for
 * its irregular rows is not seen from n and nnz).  us_per_iteration: the
 * tuned value, 0 if not tuned.  Returns 1 if a tuned shape applies, 0 if not, or
 * MW_EINVAL.
 */
int mw_cg_shape(mw_arith_t a, int32_t n, int32_t nnz, int32_t nsys, mw_shape_t *shape);

#ifdef __cplusplus
}
#endif

#endif /* MW_H */
