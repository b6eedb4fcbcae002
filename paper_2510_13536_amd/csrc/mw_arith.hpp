// mw_arith.hpp -- device-side multi-word arithmetic for gfx950.
//
// Values of the eight arithmetics (the paper's five, QTWE, QW, QQW) are register
// tuples Num<A> of K = words(A) FP64 words, w[0] the leading one.  Every
// operation below is one IEEE binary64 instruction with round-to-nearest-
// even (v_add_f64, v_mul_f64, v_fma_f64); contraction is disabled for this
// file so the compiler can neither fuse nor split them, and every intended
// fused multiply-add is an explicit __builtin_fma.
//
// Algorithms (Mukunoki & Ozaki, arXiv 2510.13536, Sec. III):
//   TwoSum (Alg. 2), QuickTwoSum (Alg. 3), TwoProdFMA (Alg. 4);
//   DW add/mul (Alg. 5, 6); QDW = DW without the closing QuickTwoSum;
//   QTW add/mul (Alg. 7, 8); VecSum3 (Alg. 9); FP64 x QTW (Alg. 10), and the
//   same zero-lower-word rule for FP64 x DW/QDW.
// TW is the QTW operation followed by a renormalisation (VecSum bottom-up,
// then VecSumErrBranch with three outputs, after Fabiano, Muller and Picot,
// 2019), because the paper uses their TW algorithms without printing them.
// QTWE is the QTW operation followed by VecSum3: normalisation after every
// operation, the other end of the placement question Sec. IV-D and VI leave
// open (the QDW counterpart is DW itself).  QTWE is not a "quasi" type for
// the solver: r gets no extra normalisation.
// QW (quadruple-word, named in Sec. I) follows the quad-double algorithms
// of Hida, Li and Bailey (ARITH 2001): the faster addition, the
// multiplication through third-order terms, their five-component
// renormalisation; FP64 x QW is that multiplication with the FP64
// operand's zero words, the exact identities dropped.  QQW (quasi
// quadruple-word, also named in Sec. I; its source is not available here)
// is read as the construction of QTW (Alg. 7, 8, 10) carried one order
// further, normalised by VecSum4 (Alg. 9 extended to four words).
// On the GPU the branches of VecSumErrBranch and of the QW renormalisation
// are resolved with selects, so a wavefront never diverges on them.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace mwk {

enum Arith : int { FP64 = 0, DW = 1, QDW = 2, TW = 3, QTW = 4, QTWE = 5, QW = 6, QQW = 7, MXDW = 8, MXQTW = 9 };

// Mixed precision (future work in Sec. VI): MXDW / MXQTW keep vectors in
// FP64 and accumulate SpMV rows and dots in DW / QTW.  base() is the
// multi-word arithmetic an arithmetic computes in (the accumulator's, for
// the mixed ones).
__host__ __device__ constexpr bool is_mixed(int a) { return a == MXDW || a == MXQTW; }
__host__ __device__ constexpr int base(int a) { return a == MXDW ? DW : (a == MXQTW ? QTW : a); }

// Words of a value (a register tuple, a scalar such as alpha or a dot).
__host__ __device__ constexpr int words(int a)
{
    return base(a) == FP64 ? 1
                           : ((base(a) == DW || base(a) == QDW) ? 2 : ((base(a) == QW || base(a) == QQW) ? 4 : 3));
}

// Words of a stored vector element (one FP64 word for the mixed types).
__host__ __device__ constexpr int vwords(int a) { return is_mixed(a) ? 1 : words(a); }

// Quasi types: r is normalised after its update in CG (Sec. IV-D).  The
// mixed types' r is FP64.
__host__ __device__ constexpr bool is_quasi(int a) { return a == QDW || a == QTW || a == QQW; }

template <int A>
struct Num {
    double w[words(A)];
};

template <int A>
__device__ __forceinline__ Num<A> zero()
{
    Num<A> z;
#pragma unroll
    for (int i = 0; i < words(A); ++i) z.w[i] = 0.0;
    return z;
}

template <int A>
__device__ __forceinline__ Num<A> promote(double a)
{
    Num<A> z = zero<A>();
    z.w[0] = a;
    return z;
}

// ---------------------------------------------------------------- EFTs

// s = fl(a + b), e = (a + b) - s exactly.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    const double x = a + b;
    const double z = x - a;
    e = (a - (x - z)) + (b - z);
    s = x;
}

// Exact when |a| >= |b|.
__device__ __forceinline__ void quick_two_sum(double a, double b, double &s, double &e)
{
    const double x = a + b;
    e = (a - x) + b;
    s = x;
}

// p = fl(a * b), e = a * b - p exactly (one FMA).
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e)
{
    const double x = a * b;
    e = __builtin_fma(a, b, -x);
    p = x;
}

// ------------------------------------------------- normalisations

// VecSum3 (Alg. 9): TwoSum of the top pair, then of the lower pair.
__device__ __forceinline__ void vec_sum3(double &c1, double &c2, double &c3)
{
    two_sum(c1, c2, c1, c2);
    two_sum(c2, c3, c2, c3);
}

// Full TW renormalisation: VecSum from the bottom word, then
// VecSumErrBranch(m = 3).  Resolving its two data-dependent branches by
// hand gives: with (t0, f1) = TwoSum(e0, e1),
//   f1 != 0:  (t1, f2) = TwoSum(f1, e2), result (t0, t1, f2);
//   f1 == 0:  (t1, f2) = TwoSum(t0, e2), result (t1, f2, 0).
__device__ __forceinline__ void tw_renorm(double &c1, double &c2, double &c3)
{
    double s, e1, e2;
    two_sum(c2, c3, s, e2);
    two_sum(c1, s, s, e1);
    // (t0, f1) = TwoSum(s, e1) of the branch step.  (s, e1) is already a
    // TwoSum result: |e1| <= ulp(s)/2 with ties rounding to even, so for
    // finite values t0 = s and f1 = e1 exactly; t0 = fl(s + e1) is still
    // formed, which also keeps the non-finite cases (where e1 is NaN) as
    // the full TwoSum gives them.
    const double t0 = s + e1;
    const double f1 = e1;
    const bool carry = (f1 != 0.0);
    double t1, f2;
    two_sum(carry ? f1 : t0, e2, t1, f2);
    c1 = carry ? t0 : t1;
    c2 = carry ? t1 : f2;
    c3 = carry ? f2 : 0.0;
}

// ---------------------------------------------- quadruple-word helpers

// (a, b, c) -> three words carrying the same exact sum (three TwoSums).
__device__ __forceinline__ void three_sum(double &a, double &b, double &c)
{
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, a, t3);
    two_sum(t2, t3, b, c);
}

// (a, b, c) -> two words; the error of the last FP64 sum is dropped.
__device__ __forceinline__ void three_sum2(double &a, double &b, double c)
{
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, a, t3);
    b = t2 + t3;
}

// QW renormalisation of five components (largest first) into four
// non-overlapping words: QuickTwoSums from the bottom word up, then from
// the top down, where a partial sum becomes the next output word whenever
// the error it leaves is nonzero (and the error carries on); the last
// partial sum fills the next free word.  The output index is per lane, so
// each word is chosen with selects.
__device__ __forceinline__ void qw_renorm(double c0, double c1, double c2, double c3, double c4, double &r0,
                                          double &r1, double &r2, double &r3)
{
    double s, t[5];
    quick_two_sum(c3, c4, s, t[4]);
    quick_two_sum(c2, s, s, t[3]);
    quick_two_sum(c1, s, s, t[2]);
    quick_two_sum(c0, s, t[0], t[1]);
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int k = 0;
    s = t[0];
#pragma unroll
    for (int i = 1; i < 5; ++i) {
        double u, e;
        quick_two_sum(s, t[i], u, e);
        const bool emit = (e != 0.0);
        b0 = (emit && k == 0) ? u : b0;
        b1 = (emit && k == 1) ? u : b1;
        b2 = (emit && k == 2) ? u : b2;
        b3 = (emit && k == 3) ? u : b3;
        s = emit ? e : u;
        k += emit ? 1 : 0;
    }
    r0 = k == 0 ? s : b0;
    r1 = k == 1 ? s : b1;
    r2 = k == 2 ? s : b2;
    r3 = k == 3 ? s : b3;
}

// VecSum4: TwoSums from the top word down (Alg. 9 extended to four words).
__device__ __forceinline__ void vec_sum4(double &c1, double &c2, double &c3, double &c4)
{
    two_sum(c1, c2, c1, c2);
    two_sum(c2, c3, c2, c3);
    two_sum(c3, c4, c3, c4);
}

template <int A>
__device__ __forceinline__ Num<A> normalise(Num<A> a)
{
    constexpr int B = base(A);
    if constexpr (B == DW || B == QDW) {
        quick_two_sum(a.w[0], a.w[1], a.w[0], a.w[1]);
    } else if constexpr (B == QTW || B == QTWE) {
        vec_sum3(a.w[0], a.w[1], a.w[2]);
    } else if constexpr (B == TW) {
        tw_renorm(a.w[0], a.w[1], a.w[2]);
    } else if constexpr (B == QW) {
        qw_renorm(a.w[0], a.w[1], a.w[2], a.w[3], 0.0, a.w[0], a.w[1], a.w[2], a.w[3]);
    } else if constexpr (B == QQW) {
        vec_sum4(a.w[0], a.w[1], a.w[2], a.w[3]);
    }
    return a;
}

// QW sum (the faster variant): word-wise TwoSums, each error carried into
// the next word by TwoSum or a three-term sum, the last order in FP64.
__device__ __forceinline__ void qw_add(const double *a, const double *b, double *c)
{
    double s0, s1, s2, s3, e0, e1, e2, e3;
    two_sum(a[0], b[0], s0, e0);
    two_sum(a[1], b[1], s1, e1);
    two_sum(a[2], b[2], s2, e2);
    two_sum(a[3], b[3], s3, e3);
    two_sum(s1, e0, s1, e0);
    three_sum(s2, e0, e1);
    three_sum2(s3, e0, e2);
    e0 = (e0 + e1) + e3;
    qw_renorm(s0, s1, s2, s3, e0, c[0], c[1], c[2], c[3]);
}

// QW product: products of order 0, 1, 2 exactly (TwoProdFMA), summed order
// by order with TwoSums; order-3 products and leftover errors in FP64.
__device__ __forceinline__ void qw_mul(const double *a, const double *b, double *c)
{
    double p0, p1, p2, p3, p4, p5, q0, q1, q2, q3, q4, q5, s0, s1, s2, t0, t1;
    two_prod(a[0], b[0], p0, q0);
    two_prod(a[0], b[1], p1, q1);
    two_prod(a[1], b[0], p2, q2);
    two_prod(a[0], b[2], p3, q3);
    two_prod(a[1], b[1], p4, q4);
    two_prod(a[2], b[0], p5, q5);
    three_sum(p1, p2, q0);
    three_sum(p2, q1, q2);
    three_sum(p3, p4, p5);
    two_sum(p2, p3, s0, t0);
    two_sum(q1, p4, s1, t1);
    s2 = q2 + p5;
    two_sum(s1, t0, s1, t0);
    s2 = s2 + (t0 + t1);
    double o3 = a[0] * b[3];
    o3 = o3 + a[1] * b[2];
    o3 = o3 + a[2] * b[1];
    o3 = o3 + a[3] * b[0];
    o3 = ((((o3 + q0) + q3) + q4) + q5);
    s1 = s1 + o3;
    qw_renorm(p0, p1, s0, s1, s2, c[0], c[1], c[2], c[3]);
}

// FP64 x QW: qw_mul with (a, 0, 0, 0), the operations on the zero words
// (exact identities) left out.
__device__ __forceinline__ void qw_dxmul(double a, const double *b, double *c)
{
    double p0, p1, p3, q0, q1, q3, u, s0, s1, t0;
    two_prod(a, b[0], p0, q0);
    two_prod(a, b[1], p1, q1);
    two_prod(a, b[2], p3, q3);
    two_sum(q0, p1, p1, u);
    two_sum(u, q1, u, q1);
    two_sum(u, p3, s0, t0);
    two_sum(q1, t0, s1, t0);
    s1 = s1 + (a * b[3] + q3);
    qw_renorm(p0, p1, s0, s1, t0, c[0], c[1], c[2], c[3]);
}

// QQW sum: Alg. 7 one order further.
__device__ __forceinline__ void qqw_add(const double *a, const double *b, double *c)
{
    double e1, e2, e3, e4, e5, e6, t;
    two_sum(a[0], b[0], c[0], e1);
    two_sum(a[1], b[1], t, e2);
    two_sum(t, e1, c[1], e3);
    two_sum(a[2], b[2], t, e4);
    two_sum(t, e2, t, e5);
    two_sum(t, e3, c[2], e6);
    c[3] = (((a[3] + b[3]) + e4) + e5) + e6;
}

// QQW product: Alg. 8 one order further (order 2 exact, order 3 in FP64).
__device__ __forceinline__ void qqw_mul(const double *a, const double *b, double *c)
{
    double e[15], t2, t3, t4, t5, t6, u;
    two_prod(a[0], b[0], c[0], e[1]);
    two_prod(a[0], b[1], t2, e[2]);
    two_prod(a[1], b[0], t3, e[3]);
    two_sum(t2, t3, u, e[4]);
    two_sum(u, e[1], c[1], e[5]);
    two_prod(a[0], b[2], t4, e[6]);
    two_prod(a[1], b[1], t5, e[7]);
    two_prod(a[2], b[0], t6, e[8]);
    two_sum(t4, t5, u, e[9]);
    two_sum(u, t6, u, e[10]);
    two_sum(u, e[2], u, e[11]);
    two_sum(u, e[3], u, e[12]);
    two_sum(u, e[4], u, e[13]);
    two_sum(u, e[5], c[2], e[14]);
    double d = __builtin_fma(a[3], b[0], e[6]) + __builtin_fma(a[2], b[1], e[7]);
    d = d + __builtin_fma(a[1], b[2], e[8]);
    d = d + __builtin_fma(a[0], b[3], e[9]);
    c[3] = ((((d + e[10]) + e[11]) + e[12]) + e[13]) + e[14];
}

// FP64 x QQW: Alg. 10 one order further.
__device__ __forceinline__ void qqw_dxmul(double a, const double *b, double *c)
{
    double e1, e2, e3, e4, e5, e6, t;
    two_prod(a, b[0], c[0], e1);
    two_prod(a, b[1], t, e2);
    two_sum(t, e1, c[1], e5);
    two_prod(a, b[2], t, e3);
    two_sum(t, e2, t, e4);
    two_sum(t, e5, c[2], e6);
    c[3] = (__builtin_fma(a, b[3], e3) + e4) + e6;
}

// ------------------------------------------------------ add / mul

template <int A>
__device__ __forceinline__ Num<A> add(const Num<A> &a, const Num<A> &b)
{
    constexpr int B = base(A);
    Num<A> c;
    if constexpr (B == FP64) {
        c.w[0] = a.w[0] + b.w[0];
    } else if constexpr (B == DW || B == QDW) {
        double s, e;
        two_sum(a.w[0], b.w[0], s, e);
        e = (e + a.w[1]) + b.w[1];
        if constexpr (B == DW) {
            quick_two_sum(s, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = s;
            c.w[1] = e;
        }
    } else if constexpr (B == QW) {
        qw_add(a.w, b.w, c.w);
    } else if constexpr (B == QQW) {
        qqw_add(a.w, b.w, c.w);
    } else {
        double e1, e2, e3, t;
        two_sum(a.w[0], b.w[0], c.w[0], e1);
        two_sum(a.w[1], b.w[1], t, e2);
        two_sum(t, e1, c.w[1], e3);
        c.w[2] = ((a.w[2] + b.w[2]) + e2) + e3;
        if constexpr (B == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (B == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
    }
    return c;
}

template <int A>
__device__ __forceinline__ Num<A> mul(const Num<A> &a, const Num<A> &b)
{
    constexpr int B = base(A);
    Num<A> c;
    if constexpr (B == FP64) {
        c.w[0] = a.w[0] * b.w[0];
    } else if constexpr (B == DW || B == QDW) {
        double p, e;
        two_prod(a.w[0], b.w[0], p, e);
        e = __builtin_fma(a.w[0], b.w[1], e);
        e = __builtin_fma(a.w[1], b.w[0], e);
        if constexpr (B == DW) {
            quick_two_sum(p, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = p;
            c.w[1] = e;
        }
    } else if constexpr (B == QW) {
        qw_mul(a.w, b.w, c.w);
    } else if constexpr (B == QQW) {
        qqw_mul(a.w, b.w, c.w);
    } else {
        double e1, e2, e3, e4, e5, t2, t3, u;
        two_prod(a.w[0], b.w[0], c.w[0], e1);
        two_prod(a.w[0], b.w[1], t2, e2);
        two_prod(a.w[1], b.w[0], t3, e3);
        two_sum(t2, t3, u, e4);
        two_sum(u, e1, c.w[1], e5);
        const double f1 = __builtin_fma(a.w[2], b.w[0], e2);
        const double f2 = __builtin_fma(a.w[1], b.w[1], e3);
        const double f3 = __builtin_fma(a.w[0], b.w[2], e4);
        c.w[2] = ((f1 + f2) + f3) + e5;
        if constexpr (B == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (B == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
    }
    return c;
}

// FP64 a times multi-word b (the FP64 operand's lower words are zero).
template <int A>
__device__ __forceinline__ Num<A> dxmul(double a, const Num<A> &b)
{
    constexpr int B = base(A);
    Num<A> c;
    if constexpr (B == FP64) {
        c.w[0] = a * b.w[0];
    } else if constexpr (B == DW || B == QDW) {
        double p, e;
        two_prod(a, b.w[0], p, e);
        e = __builtin_fma(a, b.w[1], e);
        if constexpr (B == DW) {
            quick_two_sum(p, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = p;
            c.w[1] = e;
        }
    } else if constexpr (B == QW) {
        qw_dxmul(a, b.w, c.w);
    } else if constexpr (B == QQW) {
        qqw_dxmul(a, b.w, c.w);
    } else {
        double e1, e2, e5, t;
        two_prod(a, b.w[0], c.w[0], e1);
        two_prod(a, b.w[1], t, e2);
        two_sum(t, e1, c.w[1], e5);
        c.w[2] = __builtin_fma(a, b.w[2], e2) + e5;
        if constexpr (B == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (B == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
    }
    return c;
}

template <int A>
__device__ __forceinline__ Num<A> neg(Num<A> a)
{
#pragma unroll
    for (int i = 0; i < words(A); ++i) a.w[i] = -a.w[i];
    return a;
}

// Multi-word value rounded to FP64: fl(x1 + x2), fl(x1 + fl(x2 + x3)),
// fl(x1 + fl(x2 + fl(x3 + x4))).
template <int A>
__device__ __forceinline__ double to_fp64(const Num<A> &a)
{
    if constexpr (words(A) == 1) return a.w[0];
    else if constexpr (words(A) == 2) return a.w[0] + a.w[1];
    else if constexpr (words(A) == 3) return a.w[0] + (a.w[1] + a.w[2]);
    else return a.w[0] + (a.w[1] + (a.w[2] + a.w[3]));
}

// a / b by long division with FP64 quotient digits.  Each remainder is
// formed in the arithmetic itself and normalised before its leading word
// yields the next digit; the digits are normalised at the end.
template <int A>
__device__ __forceinline__ Num<A> div(const Num<A> &a, const Num<A> &b)
{
    constexpr int B = base(A);
    if constexpr (B == FP64) {
        return promote<A>(a.w[0] / b.w[0]);
    } else {
        const double q1 = a.w[0] / b.w[0];
        Num<A> r = normalise<A>(add<A>(a, neg<A>(dxmul<A>(q1, b))));
        const double q2 = r.w[0] / b.w[0];
        Num<A> q;
        q.w[0] = q1;
        q.w[1] = q2;
        if constexpr (words(A) >= 3) {
            r = normalise<A>(add<A>(r, neg<A>(dxmul<A>(q2, b))));
            q.w[2] = r.w[0] / b.w[0];
        }
        if constexpr (words(A) == 4) {
            r = normalise<A>(add<A>(r, neg<A>(dxmul<A>(q.w[2], b))));
            q.w[3] = r.w[0] / b.w[0];
        }
        return normalise<A>(q);
    }
}

// ----------------------------------------- FP64-specific fused forms
// The FP64 solver writes every a*x + y as one fma (same as the plain
// FP64 CG it is the reference for).

// The mixed types update their FP64 vectors the same way, with the
// multi-word alpha (beta) rounded to FP64.
template <int A>
__device__ __forceinline__ Num<A> axpy_term(const Num<A> &alpha, const Num<A> &x, const Num<A> &y)
{
    // y + alpha * x
    if constexpr (A == FP64) return promote<A>(__builtin_fma(alpha.w[0], x.w[0], y.w[0]));
    else if constexpr (is_mixed(A)) return promote<A>(__builtin_fma(to_fp64<A>(alpha), x.w[0], y.w[0]));
    else return add<A>(y, mul<A>(alpha, x));
}

template <int A>
__device__ __forceinline__ Num<A> axmy_term(const Num<A> &alpha, const Num<A> &x, const Num<A> &y)
{
    // y - alpha * x
    if constexpr (A == FP64) return promote<A>(__builtin_fma(-alpha.w[0], x.w[0], y.w[0]));
    else if constexpr (is_mixed(A)) return promote<A>(__builtin_fma(-to_fp64<A>(alpha), x.w[0], y.w[0]));
    else return add<A>(y, neg<A>(mul<A>(alpha, x)));
}

// ------------------------------------------------------ word planes

// A mixed type's vector element is one FP64 word: loaded promoted, stored
// rounded to FP64.
template <int A>
__device__ __forceinline__ Num<A> load(const double *__restrict__ v, long n, long i)
{
    Num<A> r;
    if constexpr (is_mixed(A)) {
        r = promote<A>(v[i]);
    } else {
#pragma unroll
        for (int w = 0; w < words(A); ++w) r.w[w] = v[w * n + i];
    }
    return r;
}

template <int A>
__device__ __forceinline__ void store(double *__restrict__ v, long n, long i, const Num<A> &x)
{
    if constexpr (is_mixed(A)) {
        v[i] = to_fp64<A>(x);
    } else {
#pragma unroll
        for (int w = 0; w < words(A); ++w) v[w * n + i] = x.w[w];
    }
}

template <int A>
__device__ __forceinline__ Num<A> load_scalar(const double *__restrict__ s)
{
    Num<A> r;
#pragma unroll
    for (int w = 0; w < words(A); ++w) r.w[w] = s[w];
    return r;
}

template <int A>
__device__ __forceinline__ void store_scalar(double *__restrict__ s, const Num<A> &x)
{
#pragma unroll
    for (int w = 0; w < words(A); ++w) s[w] = x.w[w];
}

// Gather layout of the vector the SpMV reads (the solvers keep p in it):
// 2-word values interleaved (element i's words at v[2 i], v[2 i + 1]); 3-word
// values as interleaved leading pairs (v[2 i], v[2 i + 1]) followed by a
// plane of third words (v[2 n + i]); 4-word values as two interleaved pair
// planes (v[2 i], v[2 i + 1]; v[2 n + 2 i], v[2 n + 2 i + 1]).  A gathered element is then one wide
// load (plus one narrow one for 3 words) touching the fewest cache lines
// per wavefront: 16 + 8 bytes per lane instead of 24 at a 24-byte stride.
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int A>
__device__ __forceinline__ Num<A> load_il(const double *__restrict__ v, long n, long i)
{
    Num<A> r;
    if constexpr (is_mixed(A)) {
        r = promote<A>(v[i]);
    } else if constexpr (words(A) == 1) {
        r.w[0] = v[i];
    } else {
        const dvec2 t = *(const dvec2 *)(v + 2 * i);
        r.w[0] = t.x;
        r.w[1] = t.y;
        if constexpr (words(A) == 3) r.w[2] = v[2 * n + i];
        if constexpr (words(A) == 4) {
            const dvec2 u = *(const dvec2 *)(v + 2 * n + 2 * i);
            r.w[2] = u.x;
            r.w[3] = u.y;
        }
    }
    return r;
}

template <int A>
__device__ __forceinline__ void store_il(double *__restrict__ v, long n, long i, const Num<A> &x)
{
    if constexpr (is_mixed(A)) {
        v[i] = to_fp64<A>(x);
    } else if constexpr (words(A) == 1) {
        v[i] = x.w[0];
    } else {
        dvec2 t;
        t.x = x.w[0];
        t.y = x.w[1];
        *(dvec2 *)(v + 2 * i) = t;
        if constexpr (words(A) == 3) v[2 * n + i] = x.w[2];
        if constexpr (words(A) == 4) {
            dvec2 u;
            u.x = x.w[2];
            u.y = x.w[3];
            *(dvec2 *)(v + 2 * n + 2 * i) = u;
        }
    }
}

// Load of element i in word planes (IL = 0) or the gather layout (IL = 1).
template <int A, int IL>
__device__ __forceinline__ Num<A> load_v(const double *__restrict__ v, long n, long i)
{
    if constexpr (IL) return load_il<A>(v, n, i);
    else return load<A>(v, n, i);
}

template <int A, int IL>
__device__ __forceinline__ void store_v(double *__restrict__ v, long n, long i, const Num<A> &x)
{
    if constexpr (IL) store_il<A>(v, n, i, x);
    else store<A>(v, n, i, x);
}

// Lane-to-lane move of a whole value (wavefront of 64): lane l receives
// lane l + off; lanes whose source lies outside the wavefront keep their
// own value.
template <int A>
__device__ __forceinline__ Num<A> shfl_down(const Num<A> &v, int off)
{
    Num<A> r;
#pragma unroll
    for (int w = 0; w < words(A); ++w) r.w[w] = __shfl_down(v.w[w], off, 64);
    return r;
}

// Whole-wavefront shift by one lane (DPP wave_shl:1 / wave_shr:1, one VALU
// move per 32 bits): DIR = +1, lane l receives lane l + 1; DIR = -1, lane l
// receives lane l - 1.  The lane without a source (63, resp. 0) receives
// `edge`.  Must run with every lane active.
template <int DIR>
__device__ __forceinline__ double wave_shift1(double v, double edge)
{
    const long long bits = __double_as_longlong(v);
    constexpr int ctrl = DIR > 0 ? 0x130 : 0x138;
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), ctrl, 0xf, 0xf, false);
    const double r = __hiloint2double(hi, lo);
    const int lane = threadIdx.x & 63;
    return lane == (DIR > 0 ? 63 : 0) ? edge : r;
}

template <int DIR, int A>
__device__ __forceinline__ Num<A> wave_shift1(const Num<A> &v, const Num<A> &edge)
{
    Num<A> r;
#pragma unroll
    for (int w = 0; w < words(A); ++w) r.w[w] = wave_shift1<DIR>(v.w[w], edge.w[w]);
    return r;
}

}  // namespace mwk
