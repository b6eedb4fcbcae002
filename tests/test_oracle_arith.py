"""Pins of the CPU oracle's arithmetic against what the paper and exact
rational arithmetic fix (no GPU).

* Error-free transformations (Sec. III, Alg. 2-4): exactness invariants.
* Operation counts printed in Sec. III (FMA = 1 op): DWadd 11, DWmul 7,
  QDWadd 8, QDWmul 4, QTWadd 21, QTWmul 24, DxQTWmul 12 (Alg. 10).
* Accuracy against exact rationals (fractions.Fraction), with bounds a
  dropped term or flipped sign would break by orders of magnitude.
* Normalisation invariants: DW/TW results satisfy fl(c1+c2) = c1 (and
  fl(c2+c3) = c2); QuickTwoSum, VecSum3 and the TW renormalisation are
  error-free, so QDW carries the same exact value as DW, and TW and QTWE
  (QTW with VecSum3 after every operation) the same as QTW.
"""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from conftest import U, rand_mw

F = Fraction


def fr(planes, i):
    return sum((F(float(planes[j, i])) for j in range(planes.shape[0])), F(0))


# --------------------------------------------------------------------- EFTs

finite = st.floats(allow_nan=False, allow_infinity=False, min_value=-1e300, max_value=1e300)


@settings(max_examples=400, deadline=None)
@given(finite, finite)
def test_two_sum_error_free(a, b):
    x, y = O.eft("two_sum", np.array([a]), np.array([b]))
    assert x[0] == np.float64(a) + np.float64(b)
    assert F(a) + F(b) == F(float(x[0])) + F(float(y[0]))


@settings(max_examples=400, deadline=None)
@given(finite, finite)
def test_quick_two_sum_error_free_when_ordered(a, b):
    if abs(a) < abs(b):
        a, b = b, a
    x, y = O.eft("quick_two_sum", np.array([a]), np.array([b]))
    assert x[0] == np.float64(a) + np.float64(b)
    assert F(a) + F(b) == F(float(x[0])) + F(float(y[0]))


@settings(max_examples=400, deadline=None)
@given(st.floats(min_value=-1e150, max_value=1e150, allow_nan=False),
       st.floats(min_value=-1e150, max_value=1e150, allow_nan=False))
def test_two_prod_error_free(a, b):
    # exact when a*b does not underflow (Sec. III); skip the underflow range
    if a != 0 and b != 0 and abs(a * b) < 2.0 ** -960:
        return
    x, y = O.eft("two_prod", np.array([a]), np.array([b]))
    assert x[0] == np.float64(a) * np.float64(b)
    assert F(a) * F(b) == F(float(x[0])) + F(float(y[0]))


def test_eft_adversarial(rng):
    # huge exponent gaps, ties to even, signed zeros, subnormals
    a = np.array([1.0, 1.0, 2.0 ** 53, 1e308, 5e-324, -0.0, 0.0, 1.0 + 2 ** -52, 3.0])
    b = np.array([2.0 ** -53, 2.0 ** -200, 1.0, -1e292, 5e-324, 0.0, -0.0, 2.0 ** -53, 2.0 ** -52])
    x, y = O.eft("two_sum", a, b)
    for i in range(a.size):
        assert F(float(a[i])) + F(float(b[i])) == F(float(x[i])) + F(float(y[i]))
    assert x[0] == 1.0 and y[0] == 2.0 ** -53  # tie rounds to even
    n = 20000
    a = rng.standard_normal(n) * 2.0 ** rng.integers(-60, 60, n)
    b = rng.standard_normal(n) * 2.0 ** rng.integers(-60, 60, n)
    x, y = O.eft("two_sum", a, b)
    px, py = O.eft("two_prod", a, b)
    for i in range(0, n, 7):
        assert F(float(a[i])) + F(float(b[i])) == F(float(x[i])) + F(float(y[i]))
        assert F(float(a[i])) * F(float(b[i])) == F(float(px[i])) + F(float(py[i]))


# ---------------------------------------------------------------- op counts

@pytest.mark.parametrize("arith,op,count", [
    ("dw", "add", 11), ("dw", "mul", 7),          # Sec. III, DW text
    ("qdw", "add", 8), ("qdw", "mul", 4),         # Sec. III, QDW text
    ("qtw", "add", 21), ("qtw", "mul", 24),       # Sec. III, QTW text
    ("qtw", "dxmul", 12),                         # Alg. 10: 2 TwoProd + TwoSum + fma + add
    # QTWE: the QTW counts plus VecSum3 (Alg. 9: two TwoSums of 6 ops)
    ("qtwe", "add", 33), ("qtwe", "mul", 36), ("qtwe", "dxmul", 24),
    ("dw", "dxmul", 6), ("qdw", "dxmul", 3),      # DWmul / QDWmul minus the a2*b1 fma
    ("fp64", "add", 1), ("fp64", "mul", 1), ("fp64", "dxmul", 1),
])
def test_operation_counts(arith, op, count):
    k = O.WORDS[arith]
    u = np.array([[1.5], [2.0 ** -60], [2.0 ** -120]])[:k]
    v = np.array([[3.25], [-2.0 ** -58], [2.0 ** -115]])[:k]
    if op == "dxmul":
        u = np.array([1.5])
    _, c = O.elementwise(arith, op, u, v, count_ops=True)
    assert c == count


def test_tw_counts_are_qtw_plus_renormalisation():
    # reading: TW op = QTW op + VecSum (2 TwoSum) + VecSumErrBranch (2 TwoSum)
    u = np.array([[1.5], [2.0 ** -60], [2.0 ** -120]])
    v = np.array([[3.25], [-2.0 ** -58], [2.0 ** -115]])
    assert O.elementwise("tw", "add", u, v, count_ops=True)[1] == 21 + 24
    assert O.elementwise("tw", "mul", u, v, count_ops=True)[1] == 24 + 24


# ----------------------------------------------------------------- accuracy

N_ACC = 1500


def _rel(err, scale):
    return float(abs(err) / scale) if scale else float(abs(err))


@pytest.mark.parametrize("arith", ["dw", "qdw", "tw", "qtw", "qtwe"])
def test_add_mul_accuracy_against_exact(arith, rng):
    k = O.WORDS[arith]
    a = rand_mw(rng, k, N_ACC)
    b = rand_mw(rng, k, N_ACC)
    b[:, ::3] = -b[:, ::3]  # mixed signs, including cancellation
    s = O.elementwise(arith, "add", a, b)
    p = O.elementwise(arith, "mul", a, b)
    d = O.elementwise(arith, "dxmul", a[0], b)
    bound = 4 * U * U if k == 2 else 16 * U ** 3
    mbound = 8 * U * U if k == 2 else 32 * U ** 3
    worst_a = worst_m = worst_d = 0.0
    for i in range(N_ACC):
        A, B = fr(a, i), fr(b, i)
        worst_a = max(worst_a, _rel(fr(s, i) - (A + B), abs(A) + abs(B)))
        worst_m = max(worst_m, _rel(fr(p, i) - A * B, abs(A * B)))
        worst_d = max(worst_d, _rel(fr(d, i) - F(float(a[0, i])) * B, abs(F(float(a[0, i])) * B)))
    assert worst_a <= bound, worst_a / U ** k
    assert worst_m <= mbound, worst_m / U ** k
    assert worst_d <= mbound, worst_d / U ** k


@pytest.mark.parametrize("arith", ["dw", "qdw", "tw", "qtw", "qtwe"])
def test_div_accuracy_against_exact(arith, rng):
    k = O.WORDS[arith]
    a = rand_mw(rng, k, 600)
    b = rand_mw(rng, k, 600)
    q = O.elementwise(arith, "div", a, b)
    bound = 16 * U * U if k == 2 else 64 * U ** 3
    for i in range(600):
        ex = fr(a, i) / fr(b, i)
        assert _rel(fr(q, i) - ex, abs(ex)) <= bound


def test_fp64_ops_are_single_roundings(rng):
    a = rng.standard_normal(1000)
    b = rng.standard_normal(1000)
    assert np.array_equal(O.elementwise("fp64", "add", a, b)[0], a + b)
    assert np.array_equal(O.elementwise("fp64", "mul", a, b)[0], a * b)
    assert np.array_equal(O.elementwise("fp64", "div", a, b)[0], a / b)


def test_exact_special_cases():
    # integers and powers of two are exact in every arithmetic
    for arith in ["dw", "qdw", "tw", "qtw", "qtwe"]:
        k = O.WORDS[arith]
        a = np.zeros((k, 3))
        b = np.zeros((k, 3))
        a[0] = [3.0, -7.0, 0.5]
        b[0] = [5.0, 11.0, 0.25]
        np.testing.assert_array_equal(O.elementwise(arith, "add", a, b)[0], [8.0, 4.0, 0.75])
        np.testing.assert_array_equal(O.elementwise(arith, "mul", a, b)[0], [15.0, -77.0, 0.125])
        q = O.elementwise(arith, "div", a[:, 2:], b[:, 2:])
        assert q[0, 0] == 2.0 and np.all(q[1:, 0] == 0.0)
        for r in (O.elementwise(arith, "add", a, b), O.elementwise(arith, "mul", a, b)):
            assert np.all(r[1:] == 0.0)


def test_div_one_third_is_accurate():
    # 1/3 to 2 and 3 words: error below the format's precision
    for arith in ["dw", "qdw", "tw", "qtw", "qtwe"]:
        k = O.WORDS[arith]
        a = np.zeros((k, 1))
        b = np.zeros((k, 1))
        a[0] = 1.0
        b[0] = 3.0
        q = O.elementwise(arith, "div", a, b)
        err = abs(fr(q, 0) - F(1, 3))
        assert err <= F(1, 3) * F(2 ** (53 * k - 2)) ** -1


# ------------------------------------------------------ normalisation pins

@pytest.mark.parametrize("arith", ["dw", "tw"])
def test_non_quasi_results_are_normalised(arith, rng):
    k = O.WORDS[arith]
    a = rand_mw(rng, k, 3000, normalised=False)
    b = rand_mw(rng, k, 3000, normalised=False)
    for op in ("add", "mul", "div"):
        c = O.elementwise(arith, op, a, b)
        assert np.all(c[0] + c[1] == c[0])
        if k == 3:
            assert np.all(c[1] + c[2] == c[1])


@pytest.mark.parametrize("base,quasi", [("dw", "qdw"), ("tw", "qtw"), ("qtwe", "qtw")])
def test_normalisation_preserves_value(base, quasi, rng):
    # QuickTwoSum (on ordered pairs), VecSum3 and the TW renormalisation are
    # error-free: a quasi op and its normalised counterpart (DW, TW, or
    # QTWE: VecSum3 after every QTW op) carry the same exact value on the
    # same inputs.
    k = O.WORDS[base]
    a = rand_mw(rng, k, 800)
    b = rand_mw(rng, k, 800)
    for op in ("add", "mul", "dxmul"):
        ua = a[0] if op == "dxmul" else a
        c1 = O.elementwise(base, op, ua, b)
        c2 = O.elementwise(quasi, op, ua, b)
        for i in range(0, 800, 3):
            assert fr(c1, i) == fr(c2, i)
    q = rand_mw(rng, k, 500, normalised=False)
    nq = O.elementwise(quasi, "norm", q)
    nb = O.elementwise(base, "norm", q)
    for i in range(500):
        assert fr(nq, i) == fr(q, i)
        if base == "tw":
            assert fr(nb, i) == fr(q, i)


def test_vecsum3_reduces_overlap(rng):
    q = rand_mw(rng, 3, 2000, normalised=False)
    q[1] *= 2.0 ** 30  # heavy overlap
    n = O.elementwise("qtw", "norm", q)
    assert np.all(n[0] + n[1] == n[0])  # first TwoSum leaves a normalised top pair


def test_to_fp64_rounding(rng):
    for arith in ["dw", "tw"]:
        k = O.WORDS[arith]
        a = rand_mw(rng, k, 2000)
        r = O.elementwise(arith, "tofp64", a)
        for i in range(0, 2000, 5):
            ex = fr(a, i)
            assert abs(F(float(r[i])) - ex) <= abs(ex) * F(U) * (1 + F(2) ** -50)


def test_vecsum3_is_top_down():
    # Alg. 9 starts with TwoSum(c1, c2): with a zero leading word the other
    # two words pass through unchanged (a bottom-up sweep would merge them).
    q = np.array([[0.0, 0.0], [1.0, 3.0], [2.0 ** -40, -2.0 ** -30]])
    n = O.elementwise("qtw", "norm", q)
    np.testing.assert_array_equal(n, [[1.0, 3.0], [2.0 ** -40, -2.0 ** -30], [0.0, 0.0]])
    # and the leading output word is fl(c1 + c2)
    rng = np.random.default_rng(4)
    q = rand_mw(rng, 3, 500, normalised=False)
    n = O.elementwise("qtw", "norm", q)
    np.testing.assert_array_equal(n[0], q[0] + q[1])


def test_to_fp64_three_words_rounds_correctly_at_a_tie():
    # 1 + 2^-53 + 2^-100 lies just above the midpoint between 1 and its
    # successor: the correctly rounded result is 1 + 2^-52.
    x = np.array([[1.0], [2.0 ** -53], [2.0 ** -100]])
    assert O.elementwise("tw", "tofp64", x)[0] == 1.0 + 2.0 ** -52
    assert O.elementwise("qtw", "tofp64", x)[0] == 1.0 + 2.0 ** -52
