"""Second, independent reading of the paper's listings (Sec. III, Alg. 2-10)
in plain Python, checked bit for bit against the C oracle; likewise for the
quadruple-word formats the paper names in Sec. I (QW after Hida, Li and
Bailey; QQW as Alg. 7, 8, 10 carried one order further).

This is a cross-check against typing slips in the C code (operand order
inside the error sums, which only changes bits), not a pin on its own: the
mathematical pins live in test_oracle_arith.py.  Python float +, -, *, / are
IEEE binary64 with round-to-nearest-even; fma is the exact rational a*b + c
rounded once (float(Fraction) rounds correctly).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import rand_mw


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def two_sum(a, b):
    x = a + b
    z = x - a
    return x, (a - (x - z)) + (b - z)


def quick_two_sum(a, b):
    x = a + b
    return x, (a - x) + b


def two_prod(a, b):
    x = a * b
    return x, fma(a, b, -x)


def dw_add(a, b, quasi=False):
    s, e = two_sum(a[0], b[0])
    e = (e + a[1]) + b[1]
    return (s, e) if quasi else quick_two_sum(s, e)


def dw_mul(a, b, quasi=False):
    p, e = two_prod(a[0], b[0])
    e = fma(a[0], b[1], e)
    e = fma(a[1], b[0], e)
    return (p, e) if quasi else quick_two_sum(p, e)


def dw_dxmul(a, b, quasi=False):
    p, e = two_prod(a, b[0])
    e = fma(a, b[1], e)
    return (p, e) if quasi else quick_two_sum(p, e)


def qtw_add(a, b):
    c1, e1 = two_sum(a[0], b[0])
    c2, e2 = two_sum(a[1], b[1])
    c2, e3 = two_sum(c2, e1)
    return c1, c2, ((a[2] + b[2]) + e2) + e3


def qtw_mul(a, b):
    c1, e1 = two_prod(a[0], b[0])
    t2, e2 = two_prod(a[0], b[1])
    t3, e3 = two_prod(a[1], b[0])
    c2, e4 = two_sum(t2, t3)
    c2, e5 = two_sum(c2, e1)
    c3 = ((fma(a[2], b[0], e2) + fma(a[1], b[1], e3)) + fma(a[0], b[2], e4)) + e5
    return c1, c2, c3


def qtw_dxmul(a, b):
    c1, e1 = two_prod(a, b[0])
    c2, e2 = two_prod(a, b[1])
    c2, e5 = two_sum(c2, e1)
    return c1, c2, fma(a, b[2], e2) + e5


def vec_sum3(c):
    c1, c2 = two_sum(c[0], c[1])
    c2, c3 = two_sum(c2, c[2])
    return c1, c2, c3


def tw_renorm(c):
    s, e2 = two_sum(c[1], c[2])
    s, e1 = two_sum(c[0], s)
    e = [s, e1, e2]
    r = [0.0, 0.0, 0.0]
    j, eps = 0, e[0]
    for i in range(2):
        r[j], epsn = two_sum(eps, e[i + 1])
        if epsn != 0.0:
            j += 1
            eps = epsn
        else:
            eps = r[j]
    r[j] = eps
    return tuple(r)


# Quadruple-word (QW): Hida, Li and Bailey, "Algorithms for quad-double
# precision floating point arithmetic" (ARITH 2001): the faster addition,
# the multiplication through third-order terms, the renormalisation of
# five components.

def three_sum(a, b, c):
    """(a, b, c) -> three terms of the same exact sum."""
    u, v = two_sum(a, b)
    hi, w = two_sum(c, u)
    mid, lo = two_sum(v, w)
    return hi, mid, lo


def three_sum2(a, b, c):
    """(a, b, c) -> two terms; the lowest pair's error is dropped."""
    u, v = two_sum(a, b)
    hi, w = two_sum(c, u)
    return hi, v + w


def qw_renorm(c):
    """Five components, largest first -> four non-overlapping words."""
    t = [0.0] * 5
    s, t[4] = quick_two_sum(c[3], c[4])
    s, t[3] = quick_two_sum(c[2], s)
    s, t[2] = quick_two_sum(c[1], s)
    t[0], t[1] = quick_two_sum(c[0], s)
    out = []
    s = t[0]
    for i in range(1, 5):
        if len(out) == 4:
            break
        s, e = quick_two_sum(s, t[i])
        if e != 0.0:
            out.append(s)
            s = e
    if len(out) < 4:
        out.append(s)
    return tuple(out + [0.0] * (4 - len(out)))


def qw_add(a, b):
    s = [0.0] * 4
    e = [0.0] * 4
    for i in range(4):
        s[i], e[i] = two_sum(a[i], b[i])
    s[1], e0 = two_sum(s[1], e[0])
    s[2], e0, e1 = three_sum(s[2], e0, e[1])
    s[3], e0 = three_sum2(s[3], e0, e[2])
    return qw_renorm((s[0], s[1], s[2], s[3], (e0 + e1) + e[3]))


def qw_mul(a, b):
    p0, q0 = two_prod(a[0], b[0])
    p1, q1 = two_prod(a[0], b[1])
    p2, q2 = two_prod(a[1], b[0])
    p3, q3 = two_prod(a[0], b[2])
    p4, q4 = two_prod(a[1], b[1])
    p5, q5 = two_prod(a[2], b[0])
    p1, p2, q0 = three_sum(p1, p2, q0)
    p2, q1, q2 = three_sum(p2, q1, q2)
    p3, p4, p5 = three_sum(p3, p4, p5)
    s0, t0 = two_sum(p2, p3)
    s1, t1 = two_sum(q1, p4)
    s2 = q2 + p5
    s1, t0 = two_sum(s1, t0)
    s2 = s2 + (t0 + t1)
    third = a[0] * b[3]
    for term in (a[1] * b[2], a[2] * b[1], a[3] * b[0], q0, q3, q4, q5):
        third = third + term
    return qw_renorm((p0, p1, s0, s1 + third, s2))


def qw_dxmul(a, b):
    """The QW product with the FP64 operand's zero words, the same values
    as qw_mul((a, 0, 0, 0), b) but without the exact identities."""
    return qw_mul((a, 0.0, 0.0, 0.0), b)


# Quasi quadruple-word (QQW), read as Alg. 7, 8, 10 carried one order further.

def qqw_add(a, b):
    c1, e1 = two_sum(a[0], b[0])
    c2, e2 = two_sum(a[1], b[1])
    c2, e3 = two_sum(c2, e1)
    c3, e4 = two_sum(a[2], b[2])
    c3, e5 = two_sum(c3, e2)
    c3, e6 = two_sum(c3, e3)
    return c1, c2, c3, (((a[3] + b[3]) + e4) + e5) + e6


def qqw_mul(a, b):
    c1, e1 = two_prod(a[0], b[0])
    t2, e2 = two_prod(a[0], b[1])
    t3, e3 = two_prod(a[1], b[0])
    c2, e4 = two_sum(t2, t3)
    c2, e5 = two_sum(c2, e1)
    t4, e6 = two_prod(a[0], b[2])
    t5, e7 = two_prod(a[1], b[1])
    t6, e8 = two_prod(a[2], b[0])
    c3, e9 = two_sum(t4, t5)
    errs = [e9]
    for term in (t6, e2, e3, e4, e5):
        c3, err = two_sum(c3, term)
        errs.append(err)
    c4 = (fma(a[3], b[0], e6) + fma(a[2], b[1], e7)) + fma(a[1], b[2], e8)
    c4 = c4 + fma(a[0], b[3], errs[0])
    for err in errs[1:]:
        c4 = c4 + err
    return c1, c2, c3, c4


def qqw_dxmul(a, b):
    c1, e1 = two_prod(a, b[0])
    c2, e2 = two_prod(a, b[1])
    c2, e5 = two_sum(c2, e1)
    c3, e3 = two_prod(a, b[2])
    c3, e4 = two_sum(c3, e2)
    c3, e6 = two_sum(c3, e5)
    return c1, c2, c3, (fma(a, b[3], e3) + e4) + e6


def vec_sum4(c):
    c1, c2 = two_sum(c[0], c[1])
    c2, c3 = two_sum(c2, c[2])
    c3, c4 = two_sum(c3, c[3])
    return c1, c2, c3, c4


IMPL = {
    "dw": dict(add=dw_add, mul=dw_mul, dxmul=dw_dxmul, norm=lambda c: quick_two_sum(c[0], c[1])),
    "qdw": dict(add=lambda a, b: dw_add(a, b, True), mul=lambda a, b: dw_mul(a, b, True),
                dxmul=lambda a, b: dw_dxmul(a, b, True), norm=lambda c: quick_two_sum(c[0], c[1])),
    "qtw": dict(add=qtw_add, mul=qtw_mul, dxmul=qtw_dxmul, norm=vec_sum3),
    "tw": dict(add=lambda a, b: tw_renorm(qtw_add(a, b)), mul=lambda a, b: tw_renorm(qtw_mul(a, b)),
               dxmul=lambda a, b: tw_renorm(qtw_dxmul(a, b)), norm=tw_renorm),
    # QTW with VecSum3 after every operation
    "qtwe": dict(add=lambda a, b: vec_sum3(qtw_add(a, b)), mul=lambda a, b: vec_sum3(qtw_mul(a, b)),
                 dxmul=lambda a, b: vec_sum3(qtw_dxmul(a, b)), norm=vec_sum3),
    "qw": dict(add=qw_add, mul=qw_mul, dxmul=qw_dxmul, norm=lambda c: qw_renorm(tuple(c) + (0.0,))),
    "qqw": dict(add=qqw_add, mul=qqw_mul, dxmul=qqw_dxmul, norm=vec_sum4),
}


def div(arith, a, b):
    f = IMPL[arith]
    k = O.WORDS[arith]
    neg = lambda v: tuple(-w for w in v)  # noqa: E731
    q1 = a[0] / b[0]
    r = f["norm"](f["add"](a, neg(f["dxmul"](q1, b))))
    q2 = r[0] / b[0]
    if k == 2:
        return f["norm"]((q1, q2))
    r = f["norm"](f["add"](r, neg(f["dxmul"](q2, b))))
    q3 = r[0] / b[0]
    if k == 3:
        return f["norm"]((q1, q2, q3))
    r = f["norm"](f["add"](r, neg(f["dxmul"](q3, b))))
    q4 = r[0] / b[0]
    return f["norm"]((q1, q2, q3, q4))


@pytest.mark.parametrize("arith", ["dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw"])
@pytest.mark.parametrize("op", ["add", "mul", "dxmul", "div", "norm"])
def test_listing_bit_exact(arith, op):
    rng = np.random.default_rng(77)
    k = O.WORDS[arith]
    n = 400
    a = rand_mw(rng, k, n, normalised=False)
    b = rand_mw(rng, k, n, normalised=False)
    b[:, ::2] = -b[:, ::2]
    if op == "dxmul":
        got = O.elementwise(arith, op, a[0], b)
    elif op == "norm":
        got = O.elementwise(arith, op, a)
    else:
        got = O.elementwise(arith, op, a, b)
    for i in range(n):
        A = tuple(float(a[j, i]) for j in range(k))
        B = tuple(float(b[j, i]) for j in range(k))
        if op == "div":
            want = div(arith, A, B)
        elif op == "dxmul":
            want = IMPL[arith][op](A[0], B)
        elif op == "norm":
            want = IMPL[arith][op](A)
        else:
            want = IMPL[arith][op](A, B)
        assert tuple(float(got[j, i]) for j in range(k)) == tuple(want), (arith, op, i)
