"""Pins of the oracle's quadruple-word formats (named in Sec. I; their
algorithms are not in the paper) against exact rational arithmetic (no GPU).

* QW: the quad-double algorithms of Hida, Li and Bailey (ARITH 2001).
  Results are four non-overlapping words (fl(c_i + c_(i+1)) = c_i) within a
  small multiple of u^4 = 2^-212 of the exact sum / product / quotient; the
  FP64 x QW product is the full product with the FP64 operand's zero words
  (the exact identities dropped): the same values.
* QQW: read as the construction of QTW (Alg. 7, 8, 10) carried one order
  further, with VecSum4 (the extension of Alg. 9) as its normalisation.
  Its results may overlap; their exact values are within a small multiple
  of u^4 of the exact result on normalised inputs.  Operation counts of
  this reading: add 40, mul 72, FP64 x QQW 27, VecSum4 18.
* Both: integers and powers of two are exact, 1/3 to the format's
  precision, CG reaches errors near u^4 on a manufactured integer problem.
Parity with the QQW publication (Ozaki and Imamura) is unpinned: its text
is not available here.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import U, rand_mw
from paper_2510_13536_amd import problems as P

F = Fraction
U4 = U ** 4


def fr(planes, i):
    return sum((F(float(planes[j, i])) for j in range(planes.shape[0])), F(0))


@pytest.mark.parametrize("arith,op,count", [
    ("qqw", "add", 40), ("qqw", "mul", 72), ("qqw", "dxmul", 27), ("qqw", "norm", 18),
])
def test_qqw_operation_counts(arith, op, count):
    u = np.array([[1.5], [2.0 ** -60], [2.0 ** -120], [2.0 ** -175]])
    v = np.array([[3.25], [-2.0 ** -58], [2.0 ** -115], [-2.0 ** -170]])
    if op == "dxmul":
        _, c = O.elementwise(arith, op, np.array([1.5]), v, count_ops=True)
    elif op == "norm":
        _, c = O.elementwise(arith, op, u, count_ops=True)
    else:
        _, c = O.elementwise(arith, op, u, v, count_ops=True)
    assert c == count


@pytest.mark.parametrize("arith", ["qw", "qqw"])
def test_accuracy_against_exact(arith, rng):
    n = 1200
    a = rand_mw(rng, 4, n)
    b = rand_mw(rng, 4, n)
    b[:, ::3] = -b[:, ::3]  # mixed signs, including cancellation
    s = O.elementwise(arith, "add", a, b)
    p = O.elementwise(arith, "mul", a, b)
    d = O.elementwise(arith, "dxmul", a[0], b)
    worst = {"add": 0.0, "mul": 0.0, "dxmul": 0.0}
    for i in range(n):
        A, B = fr(a, i), fr(b, i)
        worst["add"] = max(worst["add"], float(abs(fr(s, i) - (A + B)) / (abs(A) + abs(B))))
        worst["mul"] = max(worst["mul"], float(abs(fr(p, i) - A * B) / abs(A * B)))
        D = F(float(a[0, i])) * B
        worst["dxmul"] = max(worst["dxmul"], float(abs(fr(d, i) - D) / abs(D)))
    assert worst["add"] <= 8 * U4, worst["add"] / U4
    assert worst["mul"] <= 16 * U4, worst["mul"] / U4
    assert worst["dxmul"] <= 16 * U4, worst["dxmul"] / U4


@pytest.mark.parametrize("arith", ["qw", "qqw"])
def test_div_accuracy_against_exact(arith, rng):
    a = rand_mw(rng, 4, 500)
    b = rand_mw(rng, 4, 500)
    q = O.elementwise(arith, "div", a, b)
    for i in range(500):
        ex = fr(a, i) / fr(b, i)
        assert abs(fr(q, i) - ex) <= 64 * U4 * abs(ex), i


def test_qw_results_are_non_overlapping(rng):
    a = rand_mw(rng, 4, 3000)
    b = rand_mw(rng, 4, 3000)
    b[:, ::2] = -b[:, ::2]
    for op in ("add", "mul", "div"):
        c = O.elementwise("qw", op, a, b)
        for j in range(3):
            assert np.all(c[j] + c[j + 1] == c[j]), (op, j)


def test_qw_dxmul_is_the_full_product_with_zero_words(rng):
    a = rand_mw(rng, 4, 3000, normalised=False)
    b = rand_mw(rng, 4, 3000, normalised=False)
    ap = np.zeros_like(a)
    ap[0] = a[0]
    assert np.array_equal(O.elementwise("qw", "dxmul", a[0], b), O.elementwise("qw", "mul", ap, b))


def test_qw_renormalisation_preserves_value_and_separates_words(rng):
    # components in decreasing magnitude with overlap (as the QW algorithms
    # produce them): the renormalisation is then a chain of exact
    # QuickTwoSums and keeps the exact sum
    q = rand_mw(rng, 4, 2000, normalised=False)
    n = O.elementwise("qw", "norm", q)
    for i in range(2000):
        assert fr(n, i) == fr(q, i)
    for j in range(3):
        assert np.all(n[j] + n[j + 1] == n[j])


def test_vecsum4_is_error_free_and_top_down(rng):
    q = rand_mw(rng, 4, 1500, normalised=False)
    q[1] *= 2.0 ** 20  # heavy overlap
    n = O.elementwise("qqw", "norm", q)
    for i in range(1500):
        assert fr(n, i) == fr(q, i)
    np.testing.assert_array_equal(n[0], q[0] + q[1])  # the first TwoSum is of the top pair
    z = np.array([[0.0], [1.0], [2.0 ** -40], [-2.0 ** -90]])
    np.testing.assert_array_equal(O.elementwise("qqw", "norm", z)[:, 0], [1.0, 2.0 ** -40, -2.0 ** -90, 0.0])


@pytest.mark.parametrize("arith", ["qw", "qqw"])
def test_exact_special_cases_and_one_third(arith):
    a = np.zeros((4, 3))
    b = np.zeros((4, 3))
    a[0] = [3.0, -7.0, 0.5]
    b[0] = [5.0, 11.0, 0.25]
    np.testing.assert_array_equal(O.elementwise(arith, "add", a, b)[0], [8.0, 4.0, 0.75])
    np.testing.assert_array_equal(O.elementwise(arith, "mul", a, b)[0], [15.0, -77.0, 0.125])
    for r in (O.elementwise(arith, "add", a, b), O.elementwise(arith, "mul", a, b)):
        assert np.all(r[1:] == 0.0)
    one = np.zeros((4, 1))
    three = np.zeros((4, 1))
    one[0], three[0] = 1.0, 3.0
    q = O.elementwise(arith, "div", one, three)
    assert abs(fr(q, 0) - F(1, 3)) <= F(1, 3) * F(2 ** (53 * 4 - 3)) ** -1


def test_to_fp64_four_words_is_summed_from_the_bottom():
    # fp64(x) = fl(x1 + fl(x2 + fl(x3 + x4))): 1 + 2^-53 + 2^-100 + 2^-160
    # lies above the midpoint of 1 and its successor, and the lower words
    # carry that into the last sum, which rounds up; with the third word
    # at 2^-140 the information is lost before the last sum (the reading is
    # not a correctly rounded conversion at such ties) and the tie rounds
    # to even
    x = np.array([[1.0, 1.0], [2.0 ** -53, 2.0 ** -53], [2.0 ** -100, 2.0 ** -140], [2.0 ** -160, 2.0 ** -200]])
    for arith in ("qw", "qqw"):
        np.testing.assert_array_equal(O.elementwise(arith, "tofp64", x), [1.0 + 2.0 ** -52, 1.0])


@pytest.mark.parametrize("arith", ["qw", "qqw"])
def test_cg_error_floor_near_u4(arith):
    """Integer manufactured solution on 2D Poisson 20 x 18 (b = A x* exact):
    at a tolerance below every format's reach, the error against x* falls to
    the format's floor: near u^4 |x*| for QW and QQW (TW/QTW stop near u^3)."""
    A = P.poisson2d(20, 18)
    xs = P.integer_vector(A.n, seed=4)
    b = A.matvec(xs)
    x, info = O.cg_solve(arith, A, b, tol=1e-58, maxit=400)
    assert info["status"] == "ok"
    err = max(abs(fr(x, j) - F(float(xs[j]))) for j in range(A.n))
    assert err < 1e-55 * np.abs(xs).max(), float(err)
    xt, _ = O.cg_solve("tw", A, b, tol=1e-58, maxit=400)
    assert max(abs(fr(xt, j) - F(float(xs[j]))) for j in range(A.n)) > 1e3 * err


def test_qqw_without_normalisation_breaks_down():
    """As for QDW and QTW (Sec. V-B), the quasi quadruple-word CG without the
    normalisation of r does not reach a tight tolerance; with it, it does."""
    A = P.poisson2d(20, 18)
    b = A.matvec(P.integer_vector(A.n, seed=4))
    _, ok = O.cg_solve("qqw", A, b, tol=1e-58, maxit=400)
    _, nn = O.cg_solve("qqw", A, b, tol=1e-58, maxit=400, normalise=False)
    assert ok["status"] == "ok"
    assert nn["status"] != "ok" or nn["iters"] > ok["iters"]
