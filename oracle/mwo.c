/*
 * mwo.c -- CPU oracle for Conjugate Gradient in FP64, double-word (DW),
 * quasi double-word (QDW, pair arithmetic), triple-word (TW) and quasi
 * triple-word (QTW) arithmetic, plus QTWE: QTW with VecSum3 after every
 * operation, and the quadruple-word formats QW and QQW.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP library (no headers, no helpers, no tables) and must stay that
 * way: the two are written independently from the paper so that one can
 * check the other.
 *
 * Source: Mukunoki & Ozaki, "Sparse Iterative Solvers Using High-Precision
 * Arithmetic with Quasi Multi-Word Algorithms" (arXiv 2510.13536).
 *   Sec. III, Alg. 2-4  : error-free transformations TwoSum, QuickTwoSum,
 *                         TwoProdFMA.
 *   Sec. III, Alg. 5-6  : DW addition and multiplication.
 *   Sec. III (QDW text) : QDW = DW without the closing QuickTwoSum.
 *   Sec. III, Alg. 7-8  : QTW addition and multiplication.
 *   Sec. III, Alg. 9    : VecSum3, the QTW normalisation.
 *   Sec. III, Alg. 10   : FP64 x QTW multiplication (lower words of the FP64
 *                         operand taken as zero; same rule for DW/QDW/TW).
 *   Sec. IV-A           : multi-word types; Sec. IV-B: CSR SpMV, DOT, AXPY;
 *   Sec. IV-C           : A, b in FP64, everything else in the arithmetic,
 *                         residual test in FP64;
 *   Sec. IV-D           : QDW/QTW normalise r right after its AXPY update.
 *   Sec. IV-D, VI       : normalising more often may gain accuracy at a cost;
 *                         the best frequency and placement are left open.
 *                         QTWE is the other end of that range: every QTW
 *                         operation (Alg. 7, 8, 10) is followed by VecSum3
 *                         (Alg. 9), and r gets no extra normalisation.  (For
 *                         QDW the same placement is DW itself, since QDW is
 *                         DW without the closing QuickTwoSum.)
 *   Alg. 1              : the CG iteration.
 *   Sec. VI             : mixed precision (future work): FP64 vectors with
 *                         the SpMV rows and the dots accumulated in a
 *                         multi-word arithmetic (mwo_cg_mixed_solve; with
 *                         Jacobi preconditioning, mwo_pcg_jacobi_mixed_solve).
 *   Sec. I              : quadruple-word (QW, Hida, Li and Bailey) and quasi
 *                         quadruple-word (QQW, Ozaki and Imamura) formats,
 *                         named but not given by the paper (see below).
 *
 * Readings where the paper is silent:
 *   - multi-operand sums inside one fl(...) are evaluated left to right;
 *   - TW: the paper uses the "fast" triple-word algorithms of Fabiano, Muller
 *     and Picot (2019) without printing them.  Here a TW operation is the
 *     QTW operation followed by a full renormalisation: a bottom-up VecSum
 *     then the branching VecSumErrBranch of that publication with m = 3.
 *     The result is error-free-renormalised, non-overlapping, and has the
 *     data-dependent branches the paper mentions;
 *   - division (needed by CG, not given): long division with FP64 quotient
 *     digits, the remainder formed in the arithmetic itself (see mw_div);
 *   - the FP64 residual test uses sqrt(fp64(rho)) / sqrt(fp64(b.b)) where
 *     both dots are carried out in the arithmetic;
 *   - rounding a multi-word value to FP64: fl(x1 + x2), fl(x1 + fl(x2 + x3)),
 *     fl(x1 + fl(x2 + fl(x3 + x4)));
 *   - QW: the quad-double algorithms published by Hida, Li and Bailey
 *     ("Algorithms for quad-double precision floating point arithmetic",
 *     ARITH 2001): the faster ("sloppy") addition, the multiplication that
 *     keeps every product term through the third order, and their
 *     five-component renormalisation.  The FP64 x QW product drops, from
 *     that multiplication, every operation on the FP64 operand's zero
 *     lower words that is an exact identity (the rule stated with Alg. 10);
 *   - QQW: its source is not available.  Read as the construction of QTW
 *     (Alg. 7, 8, 10) carried one order further: every word but the last
 *     formed by TwoSum/TwoProdFMA with the errors passed down one word,
 *     the last word one plain FP64 sum of its order's terms, no
 *     renormalisation; VecSum4 (three TwoSums from the top down, the
 *     extension of Alg. 9) normalises r in CG.  Parity with the QQW
 *     publication is unpinned.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * Contraction must stay off: every fused multiply-add below is an explicit
 * fma() call, and every other operation is one IEEE rounding.
 *
 * Vectors cross the ABI as "word planes": a k-word vector of length n is k
 * consecutive arrays of n doubles, plane 0 holding the leading word.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer rows than this run on one thread: every row's result is
 * the same on any number of threads, and below this size the threads cost
 * more than they save. */
#define MWO_PAR_MIN 65536

enum { MWO_FP64 = 0, MWO_DW = 1, MWO_QDW = 2, MWO_TW = 3, MWO_QTW = 4, MWO_QTWE = 5, MWO_QW = 6, MWO_QQW = 7 };

enum {
    MWO_OK = 0,
    MWO_NOT_CONVERGED = 1,
    MWO_BREAKDOWN = 2,
    MWO_EINVAL = -1
};

/* Element-wise operation codes (same numbering as the GPU library's
 * test-only element-wise entry point; the numbering is an interface, not
 * shared code). */
enum {
    OP_ADD = 0,   /* w = u + v              */
    OP_MUL = 1,   /* w = u * v              */
    OP_DXMUL = 2, /* w = u(FP64) * v        */
    OP_DIV = 3,   /* w = u / v              */
    OP_NORM = 4,  /* w = normalise(u)       */
    OP_NEG = 5,   /* w = -u                 */
    OP_TOFP64 = 6 /* w(FP64) = round(u)     */
};

/* ------------------------------------------------------------------------
 * FP64 operations.  Each is one IEEE-754 binary64 operation with
 * round-to-nearest-even.  In the op-counting build every call is counted,
 * with FMA (and a*b - c) as one operation and negation free (Sec. III).
 * ---------------------------------------------------------------------- */
#ifdef MWO_COUNT_OPS
static long long g_ops = 0;
#define COUNT_OP() (g_ops++)
#else
#define COUNT_OP() ((void)0)
#endif

static inline double f_add(double a, double b) { COUNT_OP(); return a + b; }
static inline double f_sub(double a, double b) { COUNT_OP(); return a - b; }
static inline double f_mul(double a, double b) { COUNT_OP(); return a * b; }
static inline double f_div(double a, double b) { COUNT_OP(); return a / b; }
/* a*b + c with a single rounding */
static inline double f_fma(double a, double b, double c) { COUNT_OP(); return fma(a, b, c); }
/* a*b - c with a single rounding (one operation, Sec. III) */
static inline double f_fms(double a, double b, double c) { COUNT_OP(); return fma(a, b, -c); }

/* ------------------------------------------------------------------------
 * Error-free transformations (Sec. III, Alg. 2-4)
 * ---------------------------------------------------------------------- */

/* TwoSum (Alg. 2): x = fl(a+b), y the exact rounding error, a+b = x+y. */
static inline void two_sum(double a, double b, double *x, double *y)
{
    double s = f_add(a, b);
    double z = f_sub(s, a);
    double t = f_sub(a, f_sub(s, z));
    double u = f_sub(b, z);
    *y = f_add(t, u);
    *x = s;
}

/* QuickTwoSum (Alg. 3): exact when |a| >= |b|. */
static inline void quick_two_sum(double a, double b, double *x, double *y)
{
    double s = f_add(a, b);
    *y = f_add(f_sub(a, s), b);
    *x = s;
}

/* TwoProdFMA (Alg. 4): x = fl(a*b), y = fma(a, b, -x), a*b = x+y. */
static inline void two_prod(double a, double b, double *x, double *y)
{
    double p = f_mul(a, b);
    *y = f_fms(a, b, p);
    *x = p;
}

/* ------------------------------------------------------------------------
 * Multi-word values.  w[0] is the leading word; words beyond the format's
 * width are kept at zero and never read.
 * ---------------------------------------------------------------------- */
typedef struct { double w[4]; } mwv;

static int words_of(int a)
{
    switch (a) {
    case MWO_FP64: return 1;
    case MWO_DW: case MWO_QDW: return 2;
    case MWO_TW: case MWO_QTW: case MWO_QTWE: return 3;
    case MWO_QW: case MWO_QQW: return 4;
    default: return -1;
    }
}

static inline mwv mw_make4(double a, double b, double c, double d)
{
    mwv r; r.w[0] = a; r.w[1] = b; r.w[2] = c; r.w[3] = d; return r;
}

static inline mwv mw_make(double a, double b, double c) { return mw_make4(a, b, c, 0.0); }

/* Promotion of an FP64 value: the lower words are zero. */
static inline mwv mw_promote(double a) { return mw_make(a, 0.0, 0.0); }

static inline mwv mw_load(int k, const double *v, long n, long i)
{
    mwv r = mw_make(0.0, 0.0, 0.0);
    for (int j = 0; j < k; j++) r.w[j] = v[(long)j * n + i];
    return r;
}

static inline void mw_store(int k, double *v, long n, long i, mwv x)
{
    for (int j = 0; j < k; j++) v[(long)j * n + i] = x.w[j];
}

/* ---- DW (Sec. III, Alg. 5-6) ------------------------------------------ */

/* DWadd (Alg. 5): TwoSum of the leading words, the two trailing words added
 * to the error left to right, then QuickTwoSum. */
static mwv dw_add(mwv a, mwv b)
{
    double s, e, c1, c2;
    two_sum(a.w[0], b.w[0], &s, &e);
    e = f_add(f_add(e, a.w[1]), b.w[1]);
    quick_two_sum(s, e, &c1, &c2);
    return mw_make(c1, c2, 0.0);
}

/* DWmul (Alg. 6): TwoProdFMA of the leading words, then the two cross terms
 * a1*b2 and a2*b1 folded into the error by FMA, then QuickTwoSum. */
static mwv dw_mul(mwv a, mwv b)
{
    double p, e, c1, c2;
    two_prod(a.w[0], b.w[0], &p, &e);
    e = f_fma(a.w[0], b.w[1], e);
    e = f_fma(a.w[1], b.w[0], e);
    quick_two_sum(p, e, &c1, &c2);
    return mw_make(c1, c2, 0.0);
}

/* FP64 x DW: DWmul with the FP64 operand's trailing word zero; the term
 * fma(0, b1, e) = e is an exact identity and is dropped (Sec. III, the
 * rule stated with Alg. 10). */
static mwv dw_dxmul(double a, mwv b)
{
    double p, e, c1, c2;
    two_prod(a, b.w[0], &p, &e);
    e = f_fma(a, b.w[1], e);
    quick_two_sum(p, e, &c1, &c2);
    return mw_make(c1, c2, 0.0);
}

/* ---- QDW: DW without the normalising QuickTwoSum (Sec. III) ----------- */

static mwv qdw_add(mwv a, mwv b)
{
    double s, e;
    two_sum(a.w[0], b.w[0], &s, &e);
    e = f_add(f_add(e, a.w[1]), b.w[1]);
    return mw_make(s, e, 0.0);
}

static mwv qdw_mul(mwv a, mwv b)
{
    double p, e;
    two_prod(a.w[0], b.w[0], &p, &e);
    e = f_fma(a.w[0], b.w[1], e);
    e = f_fma(a.w[1], b.w[0], e);
    return mw_make(p, e, 0.0);
}

static mwv qdw_dxmul(double a, mwv b)
{
    double p, e;
    two_prod(a, b.w[0], &p, &e);
    e = f_fma(a, b.w[1], e);
    return mw_make(p, e, 0.0);
}

/* ---- QTW (Sec. III, Alg. 7, 8, 9, 10) --------------------------------- */

/* QTWadd (Alg. 7). */
static mwv qtw_add(mwv a, mwv b)
{
    double c1, c2, c3, e1, e2, e3;
    two_sum(a.w[0], b.w[0], &c1, &e1);
    two_sum(a.w[1], b.w[1], &c2, &e2);
    two_sum(c2, e1, &c2, &e3);
    c3 = f_add(f_add(f_add(a.w[2], b.w[2]), e2), e3);
    return mw_make(c1, c2, c3);
}

/* QTWmul (Alg. 8). */
static mwv qtw_mul(mwv a, mwv b)
{
    double c1, c2, c3, e1, e2, e3, e4, e5, t2, t3;
    two_prod(a.w[0], b.w[0], &c1, &e1);
    two_prod(a.w[0], b.w[1], &t2, &e2);
    two_prod(a.w[1], b.w[0], &t3, &e3);
    two_sum(t2, t3, &c2, &e4);
    two_sum(c2, e1, &c2, &e5);
    c3 = f_add(f_add(f_add(f_fma(a.w[2], b.w[0], e2), f_fma(a.w[1], b.w[1], e3)),
                     f_fma(a.w[0], b.w[2], e4)),
               e5);
    return mw_make(c1, c2, c3);
}

/* DxQTWmul (Alg. 10): FP64 a times QTW b. */
static mwv qtw_dxmul(double a, mwv b)
{
    double c1, c2, c3, e1, e2, e5;
    two_prod(a, b.w[0], &c1, &e1);
    two_prod(a, b.w[1], &c2, &e2);
    two_sum(c2, e1, &c2, &e5);
    c3 = f_add(f_fma(a, b.w[2], e2), e5);
    return mw_make(c1, c2, c3);
}

/* VecSum3 (Alg. 9): two TwoSums from the top word down. */
static mwv vec_sum3(mwv c)
{
    double c1 = c.w[0], c2 = c.w[1], c3 = c.w[2];
    two_sum(c1, c2, &c1, &c2);
    two_sum(c2, c3, &c2, &c3);
    return mw_make(c1, c2, c3);
}

/* ---- TW (reading: QTW operation + renormalisation) --------------------- */

/* Renormalisation of three words into a non-overlapping triple:
 * (1) VecSum from the bottom word up, (2) the branching VecSumErrBranch
 * with m = 3 output words, as in Fabiano, Muller and Picot (2019).  Both
 * steps are error-free, so the exact sum is preserved. */
static mwv tw_renorm(mwv c)
{
    double e[3], s, r[3] = { 0.0, 0.0, 0.0 };
    /* VecSum, bottom-up */
    s = c.w[2];
    two_sum(c.w[1], s, &s, &e[2]);
    two_sum(c.w[0], s, &s, &e[1]);
    e[0] = s;
    /* VecSumErrBranch(e, m = 3) */
    int j = 0;
    double eps = e[0];
    for (int i = 0; i < 2; i++) {
        double rj, epsn;
        two_sum(eps, e[i + 1], &rj, &epsn);
        r[j] = rj;
        if (epsn != 0.0) {
            j++;
            eps = epsn;
        } else {
            eps = r[j];
        }
    }
    r[j] = eps;
    return mw_make(r[0], r[1], r[2]);
}

static mwv tw_add(mwv a, mwv b) { return tw_renorm(qtw_add(a, b)); }
static mwv tw_mul(mwv a, mwv b) { return tw_renorm(qtw_mul(a, b)); }
static mwv tw_dxmul(double a, mwv b) { return tw_renorm(qtw_dxmul(a, b)); }

/* ---- QTWE: every QTW operation followed by VecSum3 (Alg. 9) ------------ */

static mwv qtwe_add(mwv a, mwv b) { return vec_sum3(qtw_add(a, b)); }
static mwv qtwe_mul(mwv a, mwv b) { return vec_sum3(qtw_mul(a, b)); }
static mwv qtwe_dxmul(double a, mwv b) { return vec_sum3(qtw_dxmul(a, b)); }

/* ---- QW (Hida, Li and Bailey, ARITH 2001) ----------------------------- */

/* Three terms to three: (a, b, c) -> (s, e1, e2) with s + e1 + e2 = a + b + c
 * exactly, by three TwoSums. */
static void three_sum(double *a, double *b, double *c)
{
    double t1, t2, t3;
    two_sum(*a, *b, &t1, &t2);
    two_sum(*c, t1, a, &t3);
    two_sum(t2, t3, b, c);
}

/* Three terms to two: the same first two TwoSums, the last pair added in
 * FP64 (its error is dropped). */
static void three_sum2(double *a, double *b, double c)
{
    double t1, t2, t3;
    two_sum(*a, *b, &t1, &t2);
    two_sum(c, t1, a, &t3);
    *b = f_add(t2, t3);
}

/* Renormalisation of five overlapping components, largest first, into four
 * non-overlapping words: QuickTwoSums from the bottom up, then from the top
 * down, keeping a partial sum as an output word whenever the error it
 * leaves is nonzero, up to four words. */
static mwv qw_renorm(double c0, double c1, double c2, double c3, double c4)
{
    double t[5], s, e;
    quick_two_sum(c3, c4, &s, &t[4]);
    quick_two_sum(c2, s, &s, &t[3]);
    quick_two_sum(c1, s, &s, &t[2]);
    quick_two_sum(c0, s, &t[0], &t[1]);
    double b[4] = { 0.0, 0.0, 0.0, 0.0 };
    int k = 0;
    s = t[0];
    for (int i = 1; i < 5 && k < 4; i++) {
        quick_two_sum(s, t[i], &s, &e);
        if (e != 0.0) {
            b[k++] = s;
            s = e;
        }
    }
    if (k < 4) b[k] = s;
    return mw_make4(b[0], b[1], b[2], b[3]);
}

/* QW addition, the faster of the two published variants: word-wise
 * TwoSums, the errors carried into the next word with TwoSum / three-term
 * sums, the last order summed in FP64, then the renormalisation. */
static mwv qw_add(mwv a, mwv b)
{
    double s0, s1, s2, s3, e0, e1, e2, e3;
    two_sum(a.w[0], b.w[0], &s0, &e0);
    two_sum(a.w[1], b.w[1], &s1, &e1);
    two_sum(a.w[2], b.w[2], &s2, &e2);
    two_sum(a.w[3], b.w[3], &s3, &e3);
    two_sum(s1, e0, &s1, &e0);
    three_sum(&s2, &e0, &e1);
    three_sum2(&s3, &e0, e2);
    e0 = f_add(f_add(e0, e1), e3);
    return qw_renorm(s0, s1, s2, s3, e0);
}

/* QW multiplication: the products of orders 0, 1 and 2 (a_i b_j, i + j <= 2)
 * by TwoProdFMA, their sums by TwoSums order by order, the order-3 products
 * and the remaining order-2 errors summed in FP64, then the
 * renormalisation. */
static mwv qw_mul(mwv a, mwv b)
{
    double p0, p1, p2, p3, p4, p5, q0, q1, q2, q3, q4, q5;
    double s0, s1, s2, t0, t1;
    two_prod(a.w[0], b.w[0], &p0, &q0);
    two_prod(a.w[0], b.w[1], &p1, &q1);
    two_prod(a.w[1], b.w[0], &p2, &q2);
    two_prod(a.w[0], b.w[2], &p3, &q3);
    two_prod(a.w[1], b.w[1], &p4, &q4);
    two_prod(a.w[2], b.w[0], &p5, &q5);
    /* order 1: p1, p2 and the error q0 of order 0 */
    three_sum(&p1, &p2, &q0);
    /* order 2: (p2, q1, q2) + (p3, p4, p5) */
    three_sum(&p2, &q1, &q2);
    three_sum(&p3, &p4, &p5);
    two_sum(p2, p3, &s0, &t0);
    two_sum(q1, p4, &s1, &t1);
    s2 = f_add(q2, p5);
    two_sum(s1, t0, &s1, &t0);
    s2 = f_add(s2, f_add(t0, t1));
    /* order 3 */
    double o3 = f_mul(a.w[0], b.w[3]);
    o3 = f_add(o3, f_mul(a.w[1], b.w[2]));
    o3 = f_add(o3, f_mul(a.w[2], b.w[1]));
    o3 = f_add(o3, f_mul(a.w[3], b.w[0]));
    o3 = f_add(o3, q0);
    o3 = f_add(o3, q3);
    o3 = f_add(o3, q4);
    o3 = f_add(o3, q5);
    s1 = f_add(s1, o3);
    return qw_renorm(p0, p1, s0, s1, s2);
}

/* FP64 x QW: qw_mul with a = (a, 0, 0, 0), every operation whose operand is
 * one of the zero words and whose result is therefore exact dropped (the
 * rule stated with Alg. 10).  What remains: */
static mwv qw_dxmul(double a, mwv b)
{
    double p0, p1, p3, q0, q1, q3, s0, s1, s2, t0, u;
    two_prod(a, b.w[0], &p0, &q0);
    two_prod(a, b.w[1], &p1, &q1);
    two_prod(a, b.w[2], &p3, &q3);
    two_sum(q0, p1, &p1, &u);    /* order 1: three_sum(p1, 0, q0) */
    two_sum(u, q1, &u, &q1);     /* order 2: three_sum(u, q1, 0) */
    two_sum(u, p3, &s0, &t0);    /* (u, q1, 0) + (p3, 0, 0) */
    s1 = q1;
    two_sum(s1, t0, &s1, &t0);
    s2 = t0;
    s1 = f_add(s1, f_add(f_mul(a, b.w[3]), q3));
    return qw_renorm(p0, p1, s0, s1, s2);
}

/* ---- QQW (reading: Alg. 7, 8, 10 carried one order further) ----------- */

static mwv qqw_add(mwv a, mwv b)
{
    double c1, c2, c3, c4, e1, e2, e3, e4, e5, e6;
    two_sum(a.w[0], b.w[0], &c1, &e1);
    two_sum(a.w[1], b.w[1], &c2, &e2);
    two_sum(c2, e1, &c2, &e3);
    two_sum(a.w[2], b.w[2], &c3, &e4);
    two_sum(c3, e2, &c3, &e5);
    two_sum(c3, e3, &c3, &e6);
    c4 = f_add(f_add(f_add(f_add(a.w[3], b.w[3]), e4), e5), e6);
    return mw_make4(c1, c2, c3, c4);
}

static mwv qqw_mul(mwv a, mwv b)
{
    double c1, c2, c3, c4, t2, t3, t4, t5, t6;
    double e1, e2, e3, e4, e5, e6, e7, e8, e9, e10, e11, e12, e13, e14;
    two_prod(a.w[0], b.w[0], &c1, &e1);
    /* order 1 */
    two_prod(a.w[0], b.w[1], &t2, &e2);
    two_prod(a.w[1], b.w[0], &t3, &e3);
    two_sum(t2, t3, &c2, &e4);
    two_sum(c2, e1, &c2, &e5);
    /* order 2: the products, then the order-1 errors */
    two_prod(a.w[0], b.w[2], &t4, &e6);
    two_prod(a.w[1], b.w[1], &t5, &e7);
    two_prod(a.w[2], b.w[0], &t6, &e8);
    two_sum(t4, t5, &c3, &e9);
    two_sum(c3, t6, &c3, &e10);
    two_sum(c3, e2, &c3, &e11);
    two_sum(c3, e3, &c3, &e12);
    two_sum(c3, e4, &c3, &e13);
    two_sum(c3, e5, &c3, &e14);
    /* order 3, in FP64: each product takes one error by FMA */
    c4 = f_add(f_fma(a.w[3], b.w[0], e6), f_fma(a.w[2], b.w[1], e7));
    c4 = f_add(c4, f_fma(a.w[1], b.w[2], e8));
    c4 = f_add(c4, f_fma(a.w[0], b.w[3], e9));
    c4 = f_add(f_add(f_add(f_add(f_add(c4, e10), e11), e12), e13), e14);
    return mw_make4(c1, c2, c3, c4);
}

/* FP64 x QQW, the extension of Alg. 10. */
static mwv qqw_dxmul(double a, mwv b)
{
    double c1, c2, c3, c4, e1, e2, e3, e4, e5, e6;
    two_prod(a, b.w[0], &c1, &e1);
    two_prod(a, b.w[1], &c2, &e2);
    two_sum(c2, e1, &c2, &e5);
    two_prod(a, b.w[2], &c3, &e3);
    two_sum(c3, e2, &c3, &e4);
    two_sum(c3, e5, &c3, &e6);
    c4 = f_add(f_add(f_fma(a, b.w[3], e3), e4), e6);
    return mw_make4(c1, c2, c3, c4);
}

/* VecSum4: the four-word extension of Alg. 9, TwoSums from the top down. */
static mwv vec_sum4(mwv c)
{
    double c1 = c.w[0], c2 = c.w[1], c3 = c.w[2], c4 = c.w[3];
    two_sum(c1, c2, &c1, &c2);
    two_sum(c2, c3, &c2, &c3);
    two_sum(c3, c4, &c3, &c4);
    return mw_make4(c1, c2, c3, c4);
}

/* ---- Dispatch by arithmetic ------------------------------------------- */

static mwv mw_add(int ar, mwv a, mwv b)
{
    switch (ar) {
    case MWO_FP64: return mw_promote(f_add(a.w[0], b.w[0]));
    case MWO_DW: return dw_add(a, b);
    case MWO_QDW: return qdw_add(a, b);
    case MWO_TW: return tw_add(a, b);
    case MWO_QTWE: return qtwe_add(a, b);
    case MWO_QW: return qw_add(a, b);
    case MWO_QQW: return qqw_add(a, b);
    default: return qtw_add(a, b);
    }
}

static mwv mw_mul(int ar, mwv a, mwv b)
{
    switch (ar) {
    case MWO_FP64: return mw_promote(f_mul(a.w[0], b.w[0]));
    case MWO_DW: return dw_mul(a, b);
    case MWO_QDW: return qdw_mul(a, b);
    case MWO_TW: return tw_mul(a, b);
    case MWO_QTWE: return qtwe_mul(a, b);
    case MWO_QW: return qw_mul(a, b);
    case MWO_QQW: return qqw_mul(a, b);
    default: return qtw_mul(a, b);
    }
}

static mwv mw_dxmul(int ar, double a, mwv b)
{
    switch (ar) {
    case MWO_FP64: return mw_promote(f_mul(a, b.w[0]));
    case MWO_DW: return dw_dxmul(a, b);
    case MWO_QDW: return qdw_dxmul(a, b);
    case MWO_TW: return tw_dxmul(a, b);
    case MWO_QTWE: return qtwe_dxmul(a, b);
    case MWO_QW: return qw_dxmul(a, b);
    case MWO_QQW: return qqw_dxmul(a, b);
    default: return qtw_dxmul(a, b);
    }
}

/* Negation flips the sign of every word; it is exact. */
static mwv mw_neg(mwv a) { return mw_make4(-a.w[0], -a.w[1], -a.w[2], -a.w[3]); }

/* The normalisation each format uses: QuickTwoSum for the two-word types,
 * VecSum3 for QTW and QTWE (Sec. III / IV-D), the full renormalisation for
 * TW and QW, VecSum4 for QQW. */
static mwv mw_normalise(int ar, mwv a)
{
    double x, y;
    switch (ar) {
    case MWO_FP64: return a;
    case MWO_DW: case MWO_QDW:
        quick_two_sum(a.w[0], a.w[1], &x, &y);
        return mw_make(x, y, 0.0);
    case MWO_TW: return tw_renorm(a);
    case MWO_QW: return qw_renorm(a.w[0], a.w[1], a.w[2], a.w[3], 0.0);
    case MWO_QQW: return vec_sum4(a);
    default: return vec_sum3(a);
    }
}

/* Rounding to FP64. */
static double mw_to_fp64(int ar, mwv a)
{
    switch (words_of(ar)) {
    case 1: return a.w[0];
    case 2: return f_add(a.w[0], a.w[1]);
    case 3: return f_add(a.w[0], f_add(a.w[1], a.w[2]));
    default: return f_add(a.w[0], f_add(a.w[1], f_add(a.w[2], a.w[3])));
    }
}

/* Division a / b (needed by CG for alpha and beta; the paper gives no
 * algorithm).  Long division with FP64 quotient digits:
 *   q1 = fl(a1 / b1);  r = normalise(a - q1*b);  q2 = fl(r1 / b1);
 *   three and four words: r = normalise(r - q2*b);  q3 = fl(r1 / b1);
 *   four words: r = normalise(r - q3*b);  q4 = fl(r1 / b1);
 *   result = normalise(q1, q2[, q3[, q4]]).
 * The products q*b are FP64 x multi-word products and the subtractions are
 * additions of the negated product, all in the arithmetic itself. */
static mwv mw_div(int ar, mwv a, mwv b)
{
    int k = words_of(ar);
    if (k == 1) return mw_promote(f_div(a.w[0], b.w[0]));
    double q1 = f_div(a.w[0], b.w[0]);
    mwv r = mw_normalise(ar, mw_add(ar, a, mw_neg(mw_dxmul(ar, q1, b))));
    double q2 = f_div(r.w[0], b.w[0]);
    if (k == 2) return mw_normalise(ar, mw_make(q1, q2, 0.0));
    r = mw_normalise(ar, mw_add(ar, r, mw_neg(mw_dxmul(ar, q2, b))));
    double q3 = f_div(r.w[0], b.w[0]);
    if (k == 3) return mw_normalise(ar, mw_make(q1, q2, q3));
    r = mw_normalise(ar, mw_add(ar, r, mw_neg(mw_dxmul(ar, q3, b))));
    double q4 = f_div(r.w[0], b.w[0]);
    return mw_normalise(ar, mw_make4(q1, q2, q3, q4));
}

/* ------------------------------------------------------------------------
 * Exported: metadata
 * ---------------------------------------------------------------------- */
int mwo_words(int arith) { return words_of(arith); }

long long mwo_ops_get(void)
{
#ifdef MWO_COUNT_OPS
    return g_ops;
#else
    return -1;
#endif
}

void mwo_ops_reset(void)
{
#ifdef MWO_COUNT_OPS
    g_ops = 0;
#endif
}

int mwo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (timing only: the results do
 * not depend on it). */
void mwo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Exported: error-free transformations on arrays (for invariant tests).
 * which: 0 TwoSum, 1 QuickTwoSum, 2 TwoProdFMA.
 * ---------------------------------------------------------------------- */
int mwo_eft(int which, long n, const double *a, const double *b, double *x, double *y)
{
    if (n < 0 || which < 0 || which > 2) return MWO_EINVAL;
    for (long i = 0; i < n; i++) {
        if (which == 0) two_sum(a[i], b[i], &x[i], &y[i]);
        else if (which == 1) quick_two_sum(a[i], b[i], &x[i], &y[i]);
        else two_prod(a[i], b[i], &x[i], &y[i]);
    }
    return MWO_OK;
}

/* ------------------------------------------------------------------------
 * Exported: element-wise operations over word planes.
 *   u, v: k planes of n (u is one FP64 plane for OP_DXMUL);
 *   w   : k planes of n (one plane for OP_TOFP64).
 * ---------------------------------------------------------------------- */
int mwo_elementwise(int arith, int op, long n, const double *u, const double *v, double *w)
{
    int k = words_of(arith);
    if (k < 0 || n < 0 || op < OP_ADD || op > OP_TOFP64) return MWO_EINVAL;
    for (long i = 0; i < n; i++) {
        mwv a = (op == OP_DXMUL) ? mw_promote(u[i]) : mw_load(k, u, n, i);
        mwv b = (op <= OP_DIV) ? mw_load(k, v, n, i) : mw_promote(0.0);
        switch (op) {
        case OP_ADD: mw_store(k, w, n, i, mw_add(arith, a, b)); break;
        case OP_MUL: mw_store(k, w, n, i, mw_mul(arith, a, b)); break;
        case OP_DXMUL: mw_store(k, w, n, i, mw_dxmul(arith, a.w[0], b)); break;
        case OP_DIV: mw_store(k, w, n, i, mw_div(arith, a, b)); break;
        case OP_NORM: mw_store(k, w, n, i, mw_normalise(arith, a)); break;
        case OP_NEG: mw_store(k, w, n, i, mw_neg(a)); break;
        default: w[i] = mw_to_fp64(arith, a); break;
        }
    }
    return MWO_OK;
}

/* ------------------------------------------------------------------------
 * Exported: SpMV, DOT, AXPY (Sec. IV-B)
 * ---------------------------------------------------------------------- */

/* y = A x for an FP64 CSR matrix and a k-word x (Sec. IV-B).  Each row is
 * accumulated from zero in CSR order: acc = acc + a_ij * x_j, with the
 * product an FP64 x multi-word product.  FP64: acc = fma(a_ij, x_j, acc).
 * Rows are independent, so they may run in parallel without changing a bit. */
static void spmv_rows(int ar, long n, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const double *x, double *y)
{
    int k = words_of(ar);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        if (ar == MWO_FP64) {
            double acc = 0.0;
            for (long p = row_ptr[i]; p < row_ptr[i + 1]; p++)
                acc = f_fma(val[p], x[col[p]], acc);
            y[i] = acc;
        } else {
            mwv acc = mw_make(0.0, 0.0, 0.0);
            for (long p = row_ptr[i]; p < row_ptr[i + 1]; p++)
                acc = mw_add(ar, acc, mw_dxmul(ar, val[p], mw_load(k, x, n, col[p])));
            mw_store(k, y, n, i, acc);
        }
    }
}

int mwo_spmv(int arith, long n, const int32_t *row_ptr, const int32_t *col,
             const double *val, const double *x, double *y)
{
    if (words_of(arith) < 0 || n < 0) return MWO_EINVAL;
    spmv_rows(arith, n, row_ptr, col, val, x, y);
    return MWO_OK;
}

/* x^T y, accumulated sequentially from zero: acc = acc + x_i * y_i.
 * FP64: acc = fma(x_i, y_i, acc). */
static mwv dot_seq(int ar, long n, const double *x, const double *y)
{
    int k = words_of(ar);
    if (ar == MWO_FP64) {
        double acc = 0.0;
        for (long i = 0; i < n; i++) acc = f_fma(x[i], y[i], acc);
        return mw_promote(acc);
    }
    mwv acc = mw_make(0.0, 0.0, 0.0);
    for (long i = 0; i < n; i++)
        acc = mw_add(ar, acc, mw_mul(ar, mw_load(k, x, n, i), mw_load(k, y, n, i)));
    return acc;
}

int mwo_dot(int arith, long n, const double *x, const double *y, double *result)
{
    int k = words_of(arith);
    if (k < 0 || n < 0) return MWO_EINVAL;
    mwv d = dot_seq(arith, n, x, y);
    for (int j = 0; j < k; j++) result[j] = d.w[j];
    return MWO_OK;
}

/* y = y + alpha * x; alpha is k words.  FP64: y = fma(alpha, x, y). */
int mwo_axpy(int arith, long n, const double *alpha, const double *x, double *y)
{
    int k = words_of(arith);
    if (k < 0 || n < 0) return MWO_EINVAL;
    mwv al = mw_make4(alpha[0], k > 1 ? alpha[1] : 0.0, k > 2 ? alpha[2] : 0.0, k > 3 ? alpha[3] : 0.0);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        if (arith == MWO_FP64) y[i] = f_fma(al.w[0], x[i], y[i]);
        else mw_store(k, y, n, i, mw_add(arith, mw_load(k, y, n, i), mw_mul(arith, al, mw_load(k, x, n, i))));
    }
    return MWO_OK;
}

/* ------------------------------------------------------------------------
 * Exported: CG (Alg. 1 with Sec. IV-C and IV-D)
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t iters;
    int32_t status;
    double rel_res;  /* sqrt(fp64(rho)) / ||b|| at the last test */
    double seconds;  /* unused by the oracle (0) */
} mwo_cg_info;

/*
 * Solves A x = b from the initial x (k planes, overwritten with the result).
 *   r = b - A x;  p = r;  rho = r^T r;  nb = sqrt(fp64(b^T b))
 *   rho == 0: return, 0 iterations.
 *   loop:
 *     q = A p;  sigma = p^T q;  (sigma <= 0 or not finite: breakdown)
 *     alpha = rho / sigma
 *     x = x + alpha p;  r = r + (-(alpha q))
 *     QDW/QTW/QQW: r = normalise(r) when normalise_r = K > 0 and the iteration
 *       number (1, 2, ...) is a multiple of K; K = 1, every iteration, is
 *       Sec. IV-D; K = 0 never (the "-NN" variants of Sec. V-B); other K
 *       explore the frequency the paper leaves open (Sec. VI).  With
 *       normalise_p, p is normalised in the same iterations (after its x
 *       update): a placement variant, not the paper's
 *     rho' = r^T r;  iters++
 *     sqrt(fp64(rho')) / nb < tol: converged               (Sec. IV-C)
 *     iters == maxit: not converged
 *     beta = rho' / rho;  p = r + beta p;  rho = rho'
 * FP64 uses fma for every a*x + y.  `hist`, when non-null, receives the
 * relative residual of every iteration (maxit entries at most).
 */
int mwo_cg_solve_np(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *b, double *x, double tol,
                    int32_t maxit, int32_t normalise_r, int32_t normalise_p, mwo_cg_info *info, double *hist);

int mwo_cg_solve(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                 const double *val, const double *b, double *x, double tol,
                 int32_t maxit, int32_t normalise_r, mwo_cg_info *info, double *hist)
{
    return mwo_cg_solve_np(arith, n, row_ptr, col, val, b, x, tol, maxit, normalise_r, 0, info, hist);
}

int mwo_cg_solve_np(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *b, double *x, double tol,
                    int32_t maxit, int32_t normalise_r, int32_t normalise_p, mwo_cg_info *info, double *hist)
{
    int k = words_of(arith);
    if (k < 0 || n <= 0 || !(tol >= 0.0) || maxit < 0 || !info) return MWO_EINVAL;
    int quasi = (arith == MWO_QDW || arith == MWO_QTW || arith == MWO_QQW);
    double *r = calloc((size_t)k * n, sizeof(double));
    double *p = calloc((size_t)k * n, sizeof(double));
    double *q = calloc((size_t)k * n, sizeof(double));
    double *bw = calloc((size_t)k * n, sizeof(double));
    if (!r || !p || !q || !bw) { free(r); free(p); free(q); free(bw); return MWO_EINVAL; }
    memcpy(bw, b, sizeof(double) * n); /* b promoted: lower planes zero */

    info->iters = 0;
    info->status = MWO_OK;
    info->rel_res = 0.0;
    info->seconds = 0.0;

    /* r = b - A x */
    spmv_rows(arith, n, row_ptr, col, val, x, q);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        if (arith == MWO_FP64) r[i] = f_sub(b[i], q[i]);
        else mw_store(k, r, n, i, mw_add(arith, mw_promote(b[i]), mw_neg(mw_load(k, q, n, i))));
    }
    memcpy(p, r, sizeof(double) * k * n);
    mwv rho = dot_seq(arith, n, r, r);
    double nb = sqrt(mw_to_fp64(arith, dot_seq(arith, n, bw, bw)));
    int status = MWO_OK;

    if (mw_to_fp64(arith, rho) == 0.0) goto done;
    info->rel_res = sqrt(mw_to_fp64(arith, rho)) / nb;
    if (maxit == 0) { status = MWO_NOT_CONVERGED; goto done; }

    for (;;) {
        spmv_rows(arith, n, row_ptr, col, val, p, q);
        mwv sigma = dot_seq(arith, n, p, q);
        double s64 = mw_to_fp64(arith, sigma);
        if (!(s64 > 0.0) || !isfinite(s64)) { status = MWO_BREAKDOWN; break; }
        mwv alpha = mw_div(arith, rho, sigma);
        if (!isfinite(mw_to_fp64(arith, alpha))) { status = MWO_BREAKDOWN; break; }
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
        for (long i = 0; i < n; i++) {
            if (arith == MWO_FP64) {
                x[i] = f_fma(alpha.w[0], p[i], x[i]);
                r[i] = f_fma(-alpha.w[0], q[i], r[i]);
            } else {
                mwv pi = mw_load(k, p, n, i), qi = mw_load(k, q, n, i);
                mw_store(k, x, n, i, mw_add(arith, mw_load(k, x, n, i), mw_mul(arith, alpha, pi)));
                mwv ri = mw_add(arith, mw_load(k, r, n, i), mw_neg(mw_mul(arith, alpha, qi)));
                if (quasi && normalise_r > 0 && (info->iters + 1) % normalise_r == 0) {
                    ri = mw_normalise(arith, ri);
                    if (normalise_p) mw_store(k, p, n, i, mw_normalise(arith, pi));
                }
                mw_store(k, r, n, i, ri);
            }
        }
        mwv rho_new = dot_seq(arith, n, r, r);
        info->iters++;
        double rr = mw_to_fp64(arith, rho_new);
        if (!isfinite(rr)) { status = MWO_BREAKDOWN; break; }
        info->rel_res = sqrt(rr) / nb;
        if (hist && info->iters <= maxit) hist[info->iters - 1] = info->rel_res;
        if (info->rel_res < tol) break;
        if (info->iters >= maxit) { status = MWO_NOT_CONVERGED; break; }
        mwv beta = mw_div(arith, rho_new, rho);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
        for (long i = 0; i < n; i++) {
            if (arith == MWO_FP64) p[i] = f_fma(beta.w[0], p[i], r[i]);
            else mw_store(k, p, n, i, mw_add(arith, mw_load(k, r, n, i), mw_mul(arith, beta, mw_load(k, p, n, i))));
        }
        rho = rho_new;
    }
done:
    info->status = status;
    free(r); free(p); free(q); free(bw);
    return status;
}

/* ------------------------------------------------------------------------
 * Exported: Jacobi-preconditioned CG (an extension the paper names as
 * future work, Sec. VI; its algorithm is not in the paper)
 * ---------------------------------------------------------------------- */
/*
 * Reading: the textbook preconditioned CG with M = diag(A), where M^-1 is
 * the FP64 diagonal matrix of the rounded reciprocals d_i = fl(1 / a_ii)
 * (so multi-word arithmetic stays in the SpMV, the dots and the vector
 * updates, and the preconditioner is one FP64 x multi-word product per
 * row).  The stopping test is the paper's, on the residual r itself.
 *   r = b - A x;  z = D r (z_i = d_i x r_i, the FP64 x multi-word product);
 *   p = z;  rho = r^T z;  rr = r^T r;  nb = sqrt(fp64(b^T b))
 *   rr == 0: return, 0 iterations.
 *   loop:
 *     q = A p;  sigma = p^T q;  (sigma <= 0 or not finite: breakdown)
 *     alpha = rho / sigma
 *     x = x + alpha p;  r = r + (-(alpha q));  QDW/QTW/QQW: r = normalise(r)
 *       as in mwo_cg_solve (normalise_r = K)
 *     z = D r;  rho' = r^T z;  rr = r^T r;  iters++
 *     sqrt(fp64(rr)) / nb < tol: converged
 *     iters == maxit: not converged
 *     beta = rho' / rho;  p = z + beta p;  rho = rho'
 * A row without a stored diagonal entry, or a zero one, makes d_i
 * infinite, and the solve ends with a breakdown.  FP64 uses fma for every
 * a*x + y and one rounded product for z.
 */
static mwv jacobi_apply(int arith, double d, mwv r)
{
    if (arith == MWO_FP64) return mw_promote(f_mul(d, r.w[0]));
    return mw_dxmul(arith, d, r);
}

int mwo_pcg_jacobi_solve(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                         const double *val, const double *b, double *x, double tol,
                         int32_t maxit, int32_t normalise_r, mwo_cg_info *info, double *hist)
{
    int k = words_of(arith);
    if (k < 0 || n <= 0 || !(tol >= 0.0) || maxit < 0 || !info) return MWO_EINVAL;
    int quasi = (arith == MWO_QDW || arith == MWO_QTW || arith == MWO_QQW);
    double *r = calloc((size_t)k * n, sizeof(double));
    double *z = calloc((size_t)k * n, sizeof(double));
    double *p = calloc((size_t)k * n, sizeof(double));
    double *q = calloc((size_t)k * n, sizeof(double));
    double *bw = calloc((size_t)k * n, sizeof(double));
    double *d = calloc((size_t)n, sizeof(double));
    if (!r || !z || !p || !q || !bw || !d) {
        free(r); free(z); free(p); free(q); free(bw); free(d);
        return MWO_EINVAL;
    }
    memcpy(bw, b, sizeof(double) * n);
    for (long i = 0; i < n; i++) {
        double aii = 0.0;
        for (int32_t j = row_ptr[i]; j < row_ptr[i + 1]; j++)
            if (col[j] == i) aii = val[j];
        d[i] = f_div(1.0, aii);
    }

    info->iters = 0;
    info->status = MWO_OK;
    info->rel_res = 0.0;
    info->seconds = 0.0;

    spmv_rows(arith, n, row_ptr, col, val, x, q);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        mwv ri;
        if (arith == MWO_FP64) ri = mw_promote(f_sub(b[i], q[i]));
        else ri = mw_add(arith, mw_promote(b[i]), mw_neg(mw_load(k, q, n, i)));
        mw_store(k, r, n, i, ri);
        mw_store(k, z, n, i, jacobi_apply(arith, d[i], ri));
    }
    memcpy(p, z, sizeof(double) * k * n);
    mwv rho = dot_seq(arith, n, r, z);
    double rr = mw_to_fp64(arith, dot_seq(arith, n, r, r));
    double nb = sqrt(mw_to_fp64(arith, dot_seq(arith, n, bw, bw)));
    int status = MWO_OK;

    if (rr == 0.0) goto done;
    info->rel_res = sqrt(rr) / nb;
    if (maxit == 0) { status = MWO_NOT_CONVERGED; goto done; }

    for (;;) {
        spmv_rows(arith, n, row_ptr, col, val, p, q);
        mwv sigma = dot_seq(arith, n, p, q);
        double s64 = mw_to_fp64(arith, sigma);
        if (!(s64 > 0.0) || !isfinite(s64)) { status = MWO_BREAKDOWN; break; }
        mwv alpha = mw_div(arith, rho, sigma);
        if (!isfinite(mw_to_fp64(arith, alpha))) { status = MWO_BREAKDOWN; break; }
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
        for (long i = 0; i < n; i++) {
            mwv ri;
            if (arith == MWO_FP64) {
                x[i] = f_fma(alpha.w[0], p[i], x[i]);
                ri = mw_promote(f_fma(-alpha.w[0], q[i], r[i]));
            } else {
                mwv pi = mw_load(k, p, n, i), qi = mw_load(k, q, n, i);
                mw_store(k, x, n, i, mw_add(arith, mw_load(k, x, n, i), mw_mul(arith, alpha, pi)));
                ri = mw_add(arith, mw_load(k, r, n, i), mw_neg(mw_mul(arith, alpha, qi)));
                if (quasi && normalise_r > 0 && (info->iters + 1) % normalise_r == 0) ri = mw_normalise(arith, ri);
            }
            mw_store(k, r, n, i, ri);
            mw_store(k, z, n, i, jacobi_apply(arith, d[i], ri));
        }
        mwv rho_new = dot_seq(arith, n, r, z);
        rr = mw_to_fp64(arith, dot_seq(arith, n, r, r));
        info->iters++;
        if (!isfinite(rr) || !isfinite(mw_to_fp64(arith, rho_new))) { status = MWO_BREAKDOWN; break; }
        info->rel_res = sqrt(rr) / nb;
        if (hist && info->iters <= maxit) hist[info->iters - 1] = info->rel_res;
        if (info->rel_res < tol) break;
        if (info->iters >= maxit) { status = MWO_NOT_CONVERGED; break; }
        mwv beta = mw_div(arith, rho_new, rho);
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
        for (long i = 0; i < n; i++) {
            if (arith == MWO_FP64) p[i] = f_fma(beta.w[0], p[i], z[i]);
            else mw_store(k, p, n, i, mw_add(arith, mw_load(k, z, n, i), mw_mul(arith, beta, mw_load(k, p, n, i))));
        }
        rho = rho_new;
    }
done:
    info->status = status;
    free(r); free(z); free(p); free(q); free(bw); free(d);
    return status;
}

/* ------------------------------------------------------------------------
 * Exported: mixed-precision CG (Sec. VI names mixed precision as future
 * work; its algorithm is not in the paper)
 * ---------------------------------------------------------------------- */
/*
 * Reading: multi-word arithmetic only where values are accumulated.  x, r,
 * p and q are FP64 vectors.  Each SpMV row is accumulated from zero in CSR
 * order in the arithmetic, acc = acc + a_ij * x_j with x_j promoted (so each
 * product is exact), and rounded once to FP64.  Each dot accumulates the
 * exact products of its FP64 entries in the arithmetic and stays
 * multi-word; alpha and beta are the arithmetic's quotients of those dots,
 * rounded to FP64 for the vector updates, which are FP64 fmas.
 *   q = A x;  r = fl(b - q);  p = r;  rho = r^T r;  nb = sqrt(fp64(b^T b))
 *   rho == 0: return, 0 iterations.
 *   loop:
 *     q = A p;  sigma = p^T q;  (sigma <= 0 or not finite: breakdown)
 *     alpha = rho / sigma;  a = fp64(alpha)
 *     x = fma(a, p, x);  r = fma(-a, q, r);  rho' = r^T r;  iters++
 *     sqrt(fp64(rho')) / nb < tol: converged;  iters == maxit: not converged
 *     beta = rho' / rho;  p = fma(fp64(beta), p, r);  rho = rho'
 * x: one FP64 plane.  The arithmetic must have two or more words.
 */
static void spmv_mixed(int ar, long n, const int32_t *row_ptr, const int32_t *col, const double *val,
                       const double *x, double *y)
{
#pragma omp parallel for schedule(static) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        mwv acc = mw_make(0.0, 0.0, 0.0);
        for (long p = row_ptr[i]; p < row_ptr[i + 1]; p++)
            acc = mw_add(ar, acc, mw_dxmul(ar, val[p], mw_promote(x[col[p]])));
        y[i] = mw_to_fp64(ar, acc);
    }
}

static mwv dot_mixed(int ar, long n, const double *x, const double *y)
{
    mwv acc = mw_make(0.0, 0.0, 0.0);
    for (long i = 0; i < n; i++) acc = mw_add(ar, acc, mw_mul(ar, mw_promote(x[i]), mw_promote(y[i])));
    return acc;
}

int mwo_cg_mixed_solve(int arith, long n, const int32_t *row_ptr, const int32_t *col, const double *val,
                       const double *b, double *x, double tol, int32_t maxit, mwo_cg_info *info, double *hist)
{
    if (words_of(arith) < 2 || n <= 0 || !(tol >= 0.0) || maxit < 0 || !info) return MWO_EINVAL;
    double *r = calloc((size_t)n, sizeof(double));
    double *p = calloc((size_t)n, sizeof(double));
    double *q = calloc((size_t)n, sizeof(double));
    if (!r || !p || !q) { free(r); free(p); free(q); return MWO_EINVAL; }
    info->iters = 0;
    info->status = MWO_OK;
    info->rel_res = 0.0;
    info->seconds = 0.0;

    spmv_mixed(arith, n, row_ptr, col, val, x, q);
    for (long i = 0; i < n; i++) r[i] = f_sub(b[i], q[i]);
    memcpy(p, r, sizeof(double) * n);
    mwv rho = dot_mixed(arith, n, r, r);
    double nb = sqrt(mw_to_fp64(arith, dot_mixed(arith, n, b, b)));
    int status = MWO_OK;

    if (mw_to_fp64(arith, rho) == 0.0) goto done;
    info->rel_res = sqrt(mw_to_fp64(arith, rho)) / nb;
    if (maxit == 0) { status = MWO_NOT_CONVERGED; goto done; }

    for (;;) {
        spmv_mixed(arith, n, row_ptr, col, val, p, q);
        mwv sigma = dot_mixed(arith, n, p, q);
        double s64 = mw_to_fp64(arith, sigma);
        if (!(s64 > 0.0) || !isfinite(s64)) { status = MWO_BREAKDOWN; break; }
        double a = mw_to_fp64(arith, mw_div(arith, rho, sigma));
        if (!isfinite(a)) { status = MWO_BREAKDOWN; break; }
        for (long i = 0; i < n; i++) {
            x[i] = f_fma(a, p[i], x[i]);
            r[i] = f_fma(-a, q[i], r[i]);
        }
        mwv rho_new = dot_mixed(arith, n, r, r);
        info->iters++;
        double rr = mw_to_fp64(arith, rho_new);
        if (!isfinite(rr)) { status = MWO_BREAKDOWN; break; }
        info->rel_res = sqrt(rr) / nb;
        if (hist && info->iters <= maxit) hist[info->iters - 1] = info->rel_res;
        if (info->rel_res < tol) break;
        if (info->iters >= maxit) { status = MWO_NOT_CONVERGED; break; }
        double be = mw_to_fp64(arith, mw_div(arith, rho_new, rho));
        for (long i = 0; i < n; i++) p[i] = f_fma(be, p[i], r[i]);
        rho = rho_new;
    }
done:
    info->status = status;
    free(r); free(p); free(q);
    return status;
}

/* Jacobi-preconditioned CG with the mixed-precision vectors (the two
 * future-work items of Sec. VI together): as mwo_pcg_jacobi_solve, with
 * d_i = fl(1 / a_ii) and z = D r, but every vector in FP64, so z_i is the
 * FP64 product fl(d_i r_i); rho = r^T z and r^T r are accumulated in the
 * arithmetic (dot_mixed), alpha and beta are the multi-word quotients
 * rounded to FP64, the updates FP64 fmas (p = fma(beta, p, z)); the test is
 * on r^T r.  A zero or missing diagonal entry gives an infinite reciprocal
 * and a breakdown. */
int mwo_pcg_jacobi_mixed_solve(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                               const double *val, const double *b, double *x, double tol, int32_t maxit,
                               mwo_cg_info *info, double *hist)
{
    if (words_of(arith) < 2 || n <= 0 || !(tol >= 0.0) || maxit < 0 || !info) return MWO_EINVAL;
    double *r = calloc((size_t)n, sizeof(double));
    double *z = calloc((size_t)n, sizeof(double));
    double *p = calloc((size_t)n, sizeof(double));
    double *q = calloc((size_t)n, sizeof(double));
    double *d = calloc((size_t)n, sizeof(double));
    if (!r || !z || !p || !q || !d) { free(r); free(z); free(p); free(q); free(d); return MWO_EINVAL; }
    for (long i = 0; i < n; i++) {
        double aii = 0.0;
        for (int32_t j = row_ptr[i]; j < row_ptr[i + 1]; j++)
            if (col[j] == i) aii = val[j];
        d[i] = f_div(1.0, aii);
    }
    info->iters = 0;
    info->status = MWO_OK;
    info->rel_res = 0.0;
    info->seconds = 0.0;

    spmv_mixed(arith, n, row_ptr, col, val, x, q);
    for (long i = 0; i < n; i++) {
        r[i] = f_sub(b[i], q[i]);
        z[i] = f_mul(d[i], r[i]);
    }
    memcpy(p, z, sizeof(double) * n);
    mwv rho = dot_mixed(arith, n, r, z);
    double rr = mw_to_fp64(arith, dot_mixed(arith, n, r, r));
    double nb = sqrt(mw_to_fp64(arith, dot_mixed(arith, n, b, b)));
    int status = MWO_OK;

    if (rr == 0.0) goto done;
    info->rel_res = sqrt(rr) / nb;
    if (maxit == 0) { status = MWO_NOT_CONVERGED; goto done; }

    for (;;) {
        spmv_mixed(arith, n, row_ptr, col, val, p, q);
        mwv sigma = dot_mixed(arith, n, p, q);
        double s64 = mw_to_fp64(arith, sigma);
        if (!(s64 > 0.0) || !isfinite(s64)) { status = MWO_BREAKDOWN; break; }
        double a = mw_to_fp64(arith, mw_div(arith, rho, sigma));
        if (!isfinite(a)) { status = MWO_BREAKDOWN; break; }
        for (long i = 0; i < n; i++) {
            x[i] = f_fma(a, p[i], x[i]);
            r[i] = f_fma(-a, q[i], r[i]);
            z[i] = f_mul(d[i], r[i]);
        }
        mwv rho_new = dot_mixed(arith, n, r, z);
        rr = mw_to_fp64(arith, dot_mixed(arith, n, r, r));
        info->iters++;
        if (!isfinite(rr) || !isfinite(mw_to_fp64(arith, rho_new))) { status = MWO_BREAKDOWN; break; }
        info->rel_res = sqrt(rr) / nb;
        if (hist && info->iters <= maxit) hist[info->iters - 1] = info->rel_res;
        if (info->rel_res < tol) break;
        if (info->iters >= maxit) { status = MWO_NOT_CONVERGED; break; }
        double be = mw_to_fp64(arith, mw_div(arith, rho_new, rho));
        for (long i = 0; i < n; i++) p[i] = f_fma(be, p[i], z[i]);
        rho = rho_new;
    }
done:
    info->status = status;
    free(r); free(z); free(p); free(q); free(d);
    return status;
}

/* ------------------------------------------------------------------------
 * Exact references: a long fixed-point (Kulisch) accumulator.
 * The accumulator is a 2304-bit two's-complement integer whose least
 * significant bit weighs 2^-1152; every finite double, and every sum of up
 * to 2^60 of them, is represented exactly.  Products of two doubles are
 * added exactly as the two parts of TwoProdFMA (exact when no underflow
 * occurs).  Used to measure the error of SpMV rows and dot products.
 * ---------------------------------------------------------------------- */
#define KL 36
#define KLSB 1152
typedef struct { uint64_t l[KL]; } kacc;

static void k_clear(kacc *a) { memset(a->l, 0, sizeof(a->l)); }

static void k_add_double(kacc *a, double d)
{
    if (d == 0.0) return;
    int e;
    double m = frexp(d, &e);                 /* d = m * 2^e, 0.5 <= |m| < 1 */
    int64_t mi = (int64_t)ldexp(m, 53);      /* exact 53-bit integer */
    int sh = e - 53 + KLSB;                  /* weight of mi's bit 0 */
    uint64_t mag = (uint64_t)(mi < 0 ? -mi : mi);
    unsigned __int128 v = (unsigned __int128)mag << (sh % 64);
    int limb = sh / 64;
    uint64_t part[2] = { (uint64_t)v, (uint64_t)(v >> 64) };
    if (mi > 0) {
        unsigned __int128 carry = 0;
        for (int i = limb; i < KL; i++) {
            unsigned __int128 t = (unsigned __int128)a->l[i] + carry + (i - limb < 2 ? part[i - limb] : 0);
            a->l[i] = (uint64_t)t;
            carry = t >> 64;
            if (i - limb >= 1 && carry == 0) break;
        }
    } else {
        uint64_t borrow = 0;
        for (int i = limb; i < KL; i++) {
            uint64_t sub = (i - limb < 2 ? part[i - limb] : 0);
            uint64_t old = a->l[i];
            uint64_t t = old - sub - borrow;
            borrow = (old < sub) || (old - sub < borrow) ? 1 : 0;
            a->l[i] = t;
            if (i - limb >= 1 && borrow == 0) break;
        }
    }
}

/* Adds the exact product a*b. */
static void k_add_prod(kacc *acc, double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    k_add_double(acc, p);
    k_add_double(acc, e);
}

/* Approximate value of the accumulator as a double (relative error about
 * 2^-52; used only to report error magnitudes). */
static double k_to_double(const kacc *a)
{
    kacc t = *a;
    int neg = (int)(t.l[KL - 1] >> 63);
    if (neg) {
        uint64_t carry = 1;
        for (int i = 0; i < KL; i++) {
            uint64_t v = ~t.l[i] + carry;
            carry = (carry && v == 0) ? 1 : 0;
            t.l[i] = v;
        }
    }
    int h = KL - 1;
    while (h >= 0 && t.l[h] == 0) h--;
    if (h < 0) return 0.0;
    double s = 0.0;
    for (int i = h; i >= 0 && i >= h - 2; i--)
        s += ldexp((double)t.l[i], 64 * i - KLSB);
    return neg ? -s : s;
}

/* Exact x^T y (all word products) into the 36 limbs of `limbs`. */
int mwo_exact_dot_limbs(int arith, long n, const double *x, const double *y, uint64_t *limbs)
{
    int k = words_of(arith);
    if (k < 0 || n < 0) return MWO_EINVAL;
    kacc acc;
    k_clear(&acc);
    for (long i = 0; i < n; i++)
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++)
                k_add_prod(&acc, x[(long)a * n + i], y[(long)b * n + i]);
    memcpy(limbs, acc.l, sizeof(acc.l));
    return MWO_OK;
}

/* Exact sum of n doubles into limbs (pins the accumulator itself). */
int mwo_exact_sum_limbs(long n, const double *t, uint64_t *limbs)
{
    if (n < 0) return MWO_EINVAL;
    kacc acc;
    k_clear(&acc);
    for (long i = 0; i < n; i++) k_add_double(&acc, t[i]);
    memcpy(limbs, acc.l, sizeof(acc.l));
    return MWO_OK;
}

/* Error of a computed dot `res` (k words): abs_err = |res - x^T y| exactly
 * formed then rounded; scale = sum_i |fp64(x_i) * fp64(y_i)|. */
int mwo_dot_error(int arith, long n, const double *x, const double *y, const double *res,
                  double *abs_err, double *scale)
{
    int k = words_of(arith);
    if (k < 0 || n < 0) return MWO_EINVAL;
    kacc acc;
    k_clear(&acc);
    double sc = 0.0;
    for (long i = 0; i < n; i++) {
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++)
                k_add_prod(&acc, x[(long)a * n + i], y[(long)b * n + i]);
        sc += fabs(x[i] * y[i]);
    }
    for (int j = 0; j < k; j++) k_add_double(&acc, -res[j]);
    *abs_err = fabs(k_to_double(&acc));
    *scale = sc;
    return MWO_OK;
}

/* Per-row error of a computed SpMV y (k planes) for the rows listed in
 * `rows` (nrows of them): abs_err[t] = |y_i - (A x)_i| exactly formed, and
 * scale[t] = sum_j |a_ij * fp64(x_j)|. */
int mwo_spmv_error(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                   const double *val, const double *x, const double *y,
                   long nrows, const int64_t *rows, double *abs_err, double *scale)
{
    int k = words_of(arith);
    if (k < 0 || n < 0 || nrows < 0) return MWO_EINVAL;
#pragma omp parallel for schedule(dynamic, 64) if (nrows >= MWO_PAR_MIN)
    for (long t = 0; t < nrows; t++) {
        long i = rows[t];
        kacc acc;
        k_clear(&acc);
        double sc = 0.0;
        for (long p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
            for (int w = 0; w < k; w++) k_add_prod(&acc, val[p], x[(long)w * n + col[p]]);
            sc += fabs(val[p] * x[col[p]]);
        }
        for (int w = 0; w < k; w++) k_add_double(&acc, -y[(long)w * n + i]);
        abs_err[t] = fabs(k_to_double(&acc));
        scale[t] = sc;
    }
    return MWO_OK;
}

/* True residual of a k-word x: res[i] = b_i - (A x)_i formed exactly per row
 * and rounded to FP64; returns ||b - A x||_2 (FP64 sum of squares of the
 * rounded entries) in *norm. */
int mwo_true_residual(int arith, long n, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const double *b, const double *x, double *norm)
{
    int k = words_of(arith);
    if (k < 0 || n < 0) return MWO_EINVAL;
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s) if (n >= MWO_PAR_MIN)
    for (long i = 0; i < n; i++) {
        kacc acc;
        k_clear(&acc);
        k_add_double(&acc, b[i]);
        for (long p = row_ptr[i]; p < row_ptr[i + 1]; p++)
            for (int w = 0; w < k; w++) k_add_prod(&acc, -val[p], x[(long)w * n + col[p]]);
        double ri = k_to_double(&acc);
        s += ri * ri;
    }
    *norm = sqrt(s);
    return MWO_OK;
}
