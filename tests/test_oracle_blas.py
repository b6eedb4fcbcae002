"""Pins of the oracle's exact accumulator, SpMV, DOT and AXPY (no GPU).

* The long fixed-point accumulator equals fractions.Fraction sums exactly.
* SpMV with an integer stencil and an integer vector is exact in every
  arithmetic: the result equals the integer product, lower words zero.
* SpMV rows, dots and AXPY stay within the accumulated error bound of the
  format against exact rational results.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import U, rand_mw
from paper_2510_13536_amd import problems as P

ARITHS = ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw"]


def test_exact_sum_matches_fraction(rng):
    t = rng.standard_normal(3000) * 2.0 ** rng.integers(-1000, 1000, 3000)
    t = np.concatenate([t, -t[:1000], [5e-324, -5e-324, 1e308, 1e308, 2.0 ** -1074]])
    assert O.exact_sum(t) == sum((Fraction(float(v)) for v in t), Fraction(0))
    assert O.exact_sum(np.array([1e308] * 8)) == 8 * Fraction(1e308)
    assert O.exact_sum(np.array([])) == 0


@pytest.mark.parametrize("arith", ARITHS)
def test_exact_dot_matches_fraction(arith, rng):
    k = O.WORDS[arith]
    x = rand_mw(rng, k, 300)
    y = rand_mw(rng, k, 300)
    ex = sum((sum(Fraction(float(x[a, i])) for a in range(k)) *
              sum(Fraction(float(y[b, i])) for b in range(k)) for i in range(300)), Fraction(0))
    assert O.exact_dot(arith, x, y) == ex


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("grid", ["2d", "3d"])
def test_spmv_integer_case_is_exact(arith, grid):
    A = P.poisson2d(23, 17) if grid == "2d" else P.poisson3d(9, 7, 5)
    x = P.integer_vector(A.n, seed=7)
    y = O.spmv(arith, A, x)
    ref = A.to_scipy().astype(np.int64) @ x.astype(np.int64)
    np.testing.assert_array_equal(y[0], ref.astype(np.float64))
    assert np.all(y[1:] == 0.0)


def _spmv_bound(k, nnz_row):
    # sequential accumulation: each add and product contributes a few u^k
    return (8 * nnz_row) * (U ** k)


@pytest.mark.parametrize("arith", ARITHS)
def test_spmv_error_bound(arith, rng):
    k = O.WORDS[arith]
    A = P.banded_spd(2000, half_bw=6, seed=11, dseed=12)
    x = rand_mw(rng, k, A.n, emin=-3, emax=3)
    y = O.spmv(arith, A, x)
    err, sc = O.spmv_error(arith, A, x, y)
    assert np.all(err <= _spmv_bound(k, 13) * sc)
    if k > 1:
        assert np.max(err / sc) < 2.0 ** -100 if k == 2 else np.max(err / sc) < 2.0 ** -145


@pytest.mark.parametrize("arith", ARITHS)
def test_dot_error_bound(arith, rng):
    k = O.WORDS[arith]
    n = 3000
    x = rand_mw(rng, k, n, emin=-4, emax=4)
    y = rand_mw(rng, k, n, emin=-4, emax=4)
    d = O.dot(arith, x, y)
    err, sc = O.dot_error(arith, x, y, d)
    assert err <= 8 * n * U ** k * sc
    # a positive sum (rho = r^T r) is far tighter
    d = O.dot(arith, x, x)
    err, sc = O.dot_error(arith, x, x, d)
    assert err <= 4 * n * U ** k * sc


@pytest.mark.parametrize("arith", ARITHS)
def test_axpy_against_exact(arith, rng):
    k = O.WORDS[arith]
    n = 400
    x = rand_mw(rng, k, n)
    y = rand_mw(rng, k, n)
    alpha = rand_mw(rng, k, 1)[:, 0]
    z = O.axpy(arith, alpha, x, y)
    A = sum(Fraction(float(w)) for w in alpha)
    for i in range(n):
        X = sum(Fraction(float(x[j, i])) for j in range(k))
        Y = sum(Fraction(float(y[j, i])) for j in range(k))
        Z = sum(Fraction(float(z[j, i])) for j in range(k))
        assert abs(Z - (Y + A * X)) <= Fraction(16 * U ** k) * (abs(Y) + abs(A * X))


def test_fp64_blas_use_fma(rng):
    x = rng.standard_normal(50)
    y = rng.standard_normal(50)
    d = O.dot("fp64", x, y)[0]
    acc = 0.0
    for i in range(50):  # acc = fma(x_i, y_i, acc), written out exactly
        acc = float(Fraction(float(x[i])) * Fraction(float(y[i])) + Fraction(acc))
    assert d == acc
