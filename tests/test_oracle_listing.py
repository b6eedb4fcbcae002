"""Second, independent reading of the paper's listings (Sec. III, Alg. 2-10)
in plain Python, checked bit for bit against the C oracle.

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
    return f["norm"]((q1, q2, q3))


@pytest.mark.parametrize("arith", ["dw", "qdw", "tw", "qtw", "qtwe"])
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
