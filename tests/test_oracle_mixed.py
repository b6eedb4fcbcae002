"""Pins of the oracle's mixed-precision CG (Sec. VI names mixed precision
as future work; the reading: FP64 vectors, the SpMV rows and the dots
accumulated in a multi-word arithmetic, alpha and beta rounded to FP64 for
FP64 fma updates).  No GPU.

* A second reading in Python, written from that description on the Python
  element operations of test_oracle_listing.py, equals the C oracle bit for
  bit (x, iterations, status, residual history) on small systems.
* Finite termination: m distinct eigenvalues -> m iterations; 4 I -> one
  iteration with x = b / 4 exactly.
* The attainable accuracy is FP64's: on a manufactured integer problem the
  recursive residual reaches 1e-30 while the error against x* stays near
  1e-15, as in FP64 CG; the full DW solver reaches 1e-29 there.
* The rounded SpMV of a multi-word accumulator is correctly rounded: with
  integer data it is exact, and the first iterate matches an FP64 CG fed
  exactly rounded row sums.
* With Jacobi preconditioning (z_i = fl(d_i r_i), d_i = fl(1 / a_ii)): the
  second reading also covers it bit for bit; a power-of-two diagonal gives
  the plain solve bit for bit; the D A D scaling of the banded case is
  undone; a zero diagonal entry breaks down at once.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2510_13536_amd import problems as P
from test_oracle_listing import IMPL, div as mw_div, fma

ACC = ["dw", "qdw", "tw", "qtw", "qw"]


def to64(v):
    if len(v) == 2:
        return v[0] + v[1]
    if len(v) == 3:
        return v[0] + (v[1] + v[2])
    return v[0] + (v[1] + (v[2] + v[3]))


def reading_mixed_cg(arith, A, b, tol, maxit, jacobi=False):
    """jacobi: preconditioned CG with d_i = fl(1 / a_ii), z_i = fl(d_i r_i),
    rho = r^T z, the test on r^T r and p = fma(beta, p, z)."""
    f = IMPL[arith]
    k = O.WORDS[arith]
    zero = (0.0,) * k

    def promote(d):
        return (d,) + (0.0,) * (k - 1)

    def spmv(x):
        out = []
        for i in range(A.n):
            acc = zero
            for j in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
                acc = f["add"](acc, f["dxmul"](float(A.val[j]), promote(x[int(A.col_idx[j])])))
            out.append(to64(acc))
        return out

    def dot(u, v):
        acc = zero
        for a, c in zip(u, v):
            acc = f["add"](acc, f["mul"](promote(a), promote(c)))
        return acc

    n = A.n
    if jacobi:
        diag = [0.0] * n
        for i in range(n):
            for j in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
                if int(A.col_idx[j]) == i:
                    diag[i] = float(A.val[j])
        d = [1.0 / a if a != 0.0 else math.copysign(math.inf, a) for a in diag]

    def precond(r):
        return [d[i] * r[i] for i in range(n)] if jacobi else r

    bl = [float(v) for v in b]
    x = [0.0] * n
    q = spmv(x)
    r = [bl[i] - q[i] for i in range(n)]
    z = precond(r)
    p = list(z)
    rho = dot(r, z)
    rr = to64(dot(r, r))
    nb = math.sqrt(to64(dot(bl, bl)))
    hist = []
    if rr == 0.0:
        return np.array(x), 0, "ok", hist
    it = 0
    while True:
        q = spmv(p)
        sigma = dot(p, q)
        s64 = to64(sigma)
        if not (s64 > 0.0) or not math.isfinite(s64):
            return np.array(x), it, "breakdown", hist
        a = to64(mw_div(arith, rho, sigma))
        if not math.isfinite(a):
            return np.array(x), it, "breakdown", hist
        x = [fma(a, p[i], x[i]) for i in range(n)]
        r = [fma(-a, q[i], r[i]) for i in range(n)]
        z = precond(r)
        rho_new = dot(r, z)
        rr = to64(dot(r, r))
        it += 1
        if not math.isfinite(rr) or not math.isfinite(to64(rho_new)):
            return np.array(x), it, "breakdown", hist
        rel = math.sqrt(rr) / nb
        hist.append(rel)
        if rel < tol:
            return np.array(x), it, "ok", hist
        if it >= maxit:
            return np.array(x), it, "not_converged", hist
        be = to64(mw_div(arith, rho_new, rho))
        p = [fma(be, p[i], z[i]) for i in range(n)]
        rho = rho_new


def small_systems():
    out = {}
    A = P.poisson1d(12)
    out["poisson1d"] = (A, P.uniform(A.n, 201))
    A = P.banded_spd(24, half_bw=3, seed=203, dseed=204)
    out["banded_scaled"] = (A, A.matvec(P.uniform(A.n, 205)))
    A = P.CSR.from_scipy(sp.diags(np.array([1.0, 2.0, 3.0] * 3)))
    out["diag3"] = (A, P.uniform(A.n, 206))
    M = P.poisson2d(4).to_scipy().tolil()
    M[0, 0] = -4.0
    out["indefinite"] = (P.CSR.from_scipy(M.tocsr()), np.eye(16)[0] + 0.25)
    return out


SMALL = small_systems()


@pytest.mark.parametrize("jacobi", [False, True])
@pytest.mark.parametrize("arith", ACC)
@pytest.mark.parametrize("name", sorted(SMALL))
def test_second_reading_bit_exact(arith, name, jacobi):
    A, b = SMALL[name]
    xr, ir, sr, hr = reading_mixed_cg(arith, A, b, 1e-300, 8, jacobi=jacobi)
    xo, io = O.cg_solve(arith, A, b, tol=1e-300, maxit=8, history=True, mixed=True,
                        precond="jacobi" if jacobi else None)
    assert xo.shape == (1, A.n)
    assert (io["iters"], io["status"]) == (ir, sr)
    assert np.array_equal(np.asarray(io["history"]).view(np.uint64), np.asarray(hr).view(np.uint64))
    assert np.array_equal(xo[0].view(np.uint64), xr.view(np.uint64))


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_finite_termination(arith):
    rng = np.random.default_rng(21)
    d = np.repeat([1.0, 2.0, 3.0, 5.0, 8.0], 40)
    A = P.CSR.from_scipy(sp.diags(d).tocsr())
    b = rng.uniform(-1, 1, d.size)
    _, info = O.cg_solve(arith, A, b, tol=1e-12, mixed=True)
    assert info["status"] == "ok" and info["iters"] == 5
    A4 = P.CSR.from_scipy(sp.diags(np.full(50, 4.0)).tocsr())
    b4 = rng.uniform(-1, 1, 50)
    x, info = O.cg_solve(arith, A4, b4, tol=1e-12, mixed=True)
    assert info["iters"] == 1 and np.array_equal(x[0], b4 / 4.0)


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_accuracy_stays_fp64s(arith):
    """x is held in FP64, so the error against an exact solution cannot fall
    below FP64's level however small the recursive residual gets."""
    A = P.poisson2d(40, 30)
    xs = P.integer_vector(A.n, seed=3)
    b = A.matvec(xs)
    x, info = O.cg_solve(arith, A, b, tol=1e-30, maxit=600, mixed=True)
    assert info["status"] == "ok" and info["rel_res"] < 1e-30
    err = np.abs(x[0] - xs).max() / np.abs(xs).max()
    assert 1e-17 < err < 1e-13
    x64, i64 = O.cg_solve("fp64", A, b, tol=1e-30, maxit=600)
    err64 = np.abs(x64[0] - xs).max() / np.abs(xs).max()
    assert err < 10 * err64 and err64 < 10 * err
    xdw, _ = O.cg_solve("dw", A, b, tol=1e-30, maxit=600)
    assert np.abs((xdw[0] - xs) + xdw[1]).max() / np.abs(xs).max() < 1e-26


def test_integer_spmv_is_exact_and_first_iterate_is_fp64_cg_on_exact_rows():
    """With integer A and b the rounded multi-word row sums are exact; the
    first mixed iterate then equals FP64 arithmetic on those exact values:
    alpha = fl(rho / sigma) of exact integer dots (rho, sigma representable
    here), x1 = alpha r0."""
    A = P.poisson2d(9, 7)
    b = P.integer_vector(A.n, seed=5).astype(np.float64)
    x, info = O.cg_solve("dw", A, b, tol=0.0, maxit=1, mixed=True)
    Ai = A.to_scipy().astype(np.int64)
    bi = b.astype(np.int64)
    rho = int(bi @ bi)
    sigma = int(bi @ (Ai @ bi))
    alpha = rho / sigma  # Python float division: correctly rounded
    np.testing.assert_array_equal(x[0], np.array([fma(alpha, float(v), 0.0) for v in b]))


def test_rejects_one_word_and_p_normalisation():
    A, b = SMALL["poisson1d"]
    with pytest.raises(ValueError):
        O.cg_solve("fp64", A, b, mixed=True)
    with pytest.raises(ValueError):
        O.cg_solve("dw", A, b, mixed=True, normalise_p=True)


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_jacobi_power_of_two_diagonal_is_plain(arith):
    """Diagonal 4 or 2: z = r / 4 (or / 2) exactly and every dot, quotient
    and update of the preconditioned solve is the plain one scaled by a power
    of two, so x, the iterations and the residuals are the plain solve's."""
    for A, b in ((lambda c: (c[0], c[1]))(P.case_poisson2d_64()),
                 (P.poisson1d(300), np.random.default_rng(8).uniform(-1, 1, 300))):
        x1, i1 = O.cg_solve(arith, A, b, tol=1e-12, history=True, mixed=True)
        x2, i2 = O.cg_solve(arith, A, b, tol=1e-12, history=True, mixed=True, precond="jacobi")
        assert i1["iters"] == i2["iters"] and i1["status"] == i2["status"] == "ok"
        assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
        assert np.array_equal(i1["history"], i2["history"])


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_jacobi_undoes_diagonal_scaling_and_zero_diagonal_breaks_down(arith):
    A, b, _ = P.case_banded_illcond(n=2048)
    _, plain = O.cg_solve(arith, A, b, tol=1e-10, maxit=2000, mixed=True)
    x, pc = O.cg_solve(arith, A, b, tol=1e-10, maxit=2000, mixed=True, precond="jacobi")
    assert plain["status"] == "not_converged"
    assert pc["status"] == "ok" and pc["iters"] <= 40
    assert O.true_residual("fp64", A, b, x) / np.linalg.norm(b) < 1e-9
    M = P.CSR.from_scipy(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]])))
    _, info = O.cg_solve(arith, M, np.array([1.0, 1.0]), mixed=True, precond="jacobi")
    assert info["status"] == "breakdown" and info["iters"] == 0
