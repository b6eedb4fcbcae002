// mw_arith.hpp -- device-side multi-word arithmetic for gfx950.
//
// Values of the six arithmetics (the paper's five and QTWE) are register
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
// On the GPU the branch of VecSumErrBranch is resolved with selects, so a
// wavefront never diverges on it.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace mwk {

enum Arith : int { FP64 = 0, DW = 1, QDW = 2, TW = 3, QTW = 4, QTWE = 5 };

__host__ __device__ constexpr int words(int a)
{
    return a == FP64 ? 1 : ((a == DW || a == QDW) ? 2 : 3);
}

__host__ __device__ constexpr bool is_quasi(int a) { return a == QDW || a == QTW; }

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

template <int A>
__device__ __forceinline__ Num<A> normalise(Num<A> a)
{
    if constexpr (A == DW || A == QDW) {
        quick_two_sum(a.w[0], a.w[1], a.w[0], a.w[1]);
    } else if constexpr (A == QTW || A == QTWE) {
        vec_sum3(a.w[0], a.w[1], a.w[2]);
    } else if constexpr (A == TW) {
        tw_renorm(a.w[0], a.w[1], a.w[2]);
    }
    return a;
}

// ------------------------------------------------------ add / mul

template <int A>
__device__ __forceinline__ Num<A> add(const Num<A> &a, const Num<A> &b)
{
    Num<A> c;
    if constexpr (A == FP64) {
        c.w[0] = a.w[0] + b.w[0];
    } else if constexpr (A == DW || A == QDW) {
        double s, e;
        two_sum(a.w[0], b.w[0], s, e);
        e = (e + a.w[1]) + b.w[1];
        if constexpr (A == DW) {
            quick_two_sum(s, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = s;
            c.w[1] = e;
        }
    } else {
        double e1, e2, e3, t;
        two_sum(a.w[0], b.w[0], c.w[0], e1);
        two_sum(a.w[1], b.w[1], t, e2);
        two_sum(t, e1, c.w[1], e3);
        c.w[2] = ((a.w[2] + b.w[2]) + e2) + e3;
        if constexpr (A == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (A == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
    }
    return c;
}

template <int A>
__device__ __forceinline__ Num<A> mul(const Num<A> &a, const Num<A> &b)
{
    Num<A> c;
    if constexpr (A == FP64) {
        c.w[0] = a.w[0] * b.w[0];
    } else if constexpr (A == DW || A == QDW) {
        double p, e;
        two_prod(a.w[0], b.w[0], p, e);
        e = __builtin_fma(a.w[0], b.w[1], e);
        e = __builtin_fma(a.w[1], b.w[0], e);
        if constexpr (A == DW) {
            quick_two_sum(p, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = p;
            c.w[1] = e;
        }
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
        if constexpr (A == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (A == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
    }
    return c;
}

// FP64 a times multi-word b (the FP64 operand's lower words are zero).
template <int A>
__device__ __forceinline__ Num<A> dxmul(double a, const Num<A> &b)
{
    Num<A> c;
    if constexpr (A == FP64) {
        c.w[0] = a * b.w[0];
    } else if constexpr (A == DW || A == QDW) {
        double p, e;
        two_prod(a, b.w[0], p, e);
        e = __builtin_fma(a, b.w[1], e);
        if constexpr (A == DW) {
            quick_two_sum(p, e, c.w[0], c.w[1]);
        } else {
            c.w[0] = p;
            c.w[1] = e;
        }
    } else {
        double e1, e2, e5, t;
        two_prod(a, b.w[0], c.w[0], e1);
        two_prod(a, b.w[1], t, e2);
        two_sum(t, e1, c.w[1], e5);
        c.w[2] = __builtin_fma(a, b.w[2], e2) + e5;
        if constexpr (A == TW) tw_renorm(c.w[0], c.w[1], c.w[2]);
        if constexpr (A == QTWE) vec_sum3(c.w[0], c.w[1], c.w[2]);
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

// Multi-word value rounded to FP64: fl(x1 + x2), fl(x1 + fl(x2 + x3)).
template <int A>
__device__ __forceinline__ double to_fp64(const Num<A> &a)
{
    if constexpr (words(A) == 1) return a.w[0];
    else if constexpr (words(A) == 2) return a.w[0] + a.w[1];
    else return a.w[0] + (a.w[1] + a.w[2]);
}

// a / b by long division with FP64 quotient digits.  Each remainder is
// formed in the arithmetic itself and normalised before its leading word
// yields the next digit; the digits are normalised at the end.
template <int A>
__device__ __forceinline__ Num<A> div(const Num<A> &a, const Num<A> &b)
{
    if constexpr (A == FP64) {
        return promote<A>(a.w[0] / b.w[0]);
    } else {
        const double q1 = a.w[0] / b.w[0];
        Num<A> r = normalise<A>(add<A>(a, neg<A>(dxmul<A>(q1, b))));
        const double q2 = r.w[0] / b.w[0];
        Num<A> q;
        q.w[0] = q1;
        q.w[1] = q2;
        if constexpr (words(A) == 3) {
            r = normalise<A>(add<A>(r, neg<A>(dxmul<A>(q2, b))));
            q.w[2] = r.w[0] / b.w[0];
        }
        return normalise<A>(q);
    }
}

// ----------------------------------------- FP64-specific fused forms
// The FP64 solver writes every a*x + y as one fma (same as the plain
// FP64 CG it is the reference for).

template <int A>
__device__ __forceinline__ Num<A> axpy_term(const Num<A> &alpha, const Num<A> &x, const Num<A> &y)
{
    // y + alpha * x
    if constexpr (A == FP64) return promote<A>(__builtin_fma(alpha.w[0], x.w[0], y.w[0]));
    else return add<A>(y, mul<A>(alpha, x));
}

template <int A>
__device__ __forceinline__ Num<A> axmy_term(const Num<A> &alpha, const Num<A> &x, const Num<A> &y)
{
    // y - alpha * x
    if constexpr (A == FP64) return promote<A>(__builtin_fma(-alpha.w[0], x.w[0], y.w[0]));
    else return add<A>(y, neg<A>(mul<A>(alpha, x)));
}

// ------------------------------------------------------ word planes

template <int A>
__device__ __forceinline__ Num<A> load(const double *__restrict__ v, long n, long i)
{
    Num<A> r;
#pragma unroll
    for (int w = 0; w < words(A); ++w) r.w[w] = v[w * n + i];
    return r;
}

template <int A>
__device__ __forceinline__ void store(double *__restrict__ v, long n, long i, const Num<A> &x)
{
#pragma unroll
    for (int w = 0; w < words(A); ++w) v[w * n + i] = x.w[w];
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
// plane of third words (v[2 n + i]).  A gathered element is then one wide
// load (plus one narrow one for 3 words) touching the fewest cache lines
// per wavefront: 16 + 8 bytes per lane instead of 24 at a 24-byte stride.
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int A>
__device__ __forceinline__ Num<A> load_il(const double *__restrict__ v, long n, long i)
{
    Num<A> r;
    if constexpr (words(A) == 1) {
        r.w[0] = v[i];
    } else {
        const dvec2 t = *(const dvec2 *)(v + 2 * i);
        r.w[0] = t.x;
        r.w[1] = t.y;
        if constexpr (words(A) == 3) r.w[2] = v[2 * n + i];
    }
    return r;
}

template <int A>
__device__ __forceinline__ void store_il(double *__restrict__ v, long n, long i, const Num<A> &x)
{
    if constexpr (words(A) == 1) {
        v[i] = x.w[0];
    } else {
        dvec2 t;
        t.x = x.w[0];
        t.y = x.w[1];
        *(dvec2 *)(v + 2 * i) = t;
        if constexpr (words(A) == 3) v[2 * n + i] = x.w[2];
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
