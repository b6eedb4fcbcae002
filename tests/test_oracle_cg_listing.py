"""Second, independent reading of the CG iteration (Alg. 1, with the FP64
residual test of Sec. IV-C and the normalisation of r of Sec. IV-D) in
plain Python, checked bit for bit against the C oracle's solver: the final
x (every word plane), the iteration count, the status and the relative
residual of every iteration.  Also the Jacobi-preconditioned form (the
textbook preconditioned CG with M^-1 = diag(fl(1/a_ii)); preconditioning is
future work in Sec. VI) and the normalise-every-K schedule (K = 0 is the
"-NN" variant of Sec. V-B).

The element operations are the Python reading of Sec. III in
test_oracle_listing.py (Fraction-based fma, native binary64 +, -, *, /).
The iteration below is written from Alg. 1 and the readings the oracle
documents, not from the C code:
  * the first pass uses p0 and rho0 (Alg. 1's loop index starts at 1);
    #iter counts the SpMVs inside the loop; rho0 = 0 stops at once;
  * operand order x <- x + alpha p, r <- r + (-(alpha q)),
    p <- r + beta p, row sum acc <- acc + a_ij x_j, dot acc <- acc + x_i y_i
    (FP64: each one fma);
  * QDW/QTW normalise r right after its update, before rho' is formed;
  * the test is sqrt(fp64(rho')) / sqrt(fp64(b^T b)) < tol;
  * breakdown when fp64(p^T q) <= 0 or is not finite, or a non-finite
    alpha or rho'.
Small systems only (n <= 30, <= 8 iterations): the Fraction fma is slow.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2510_13536_amd import problems as P
from test_oracle_listing import IMPL, div as mw_div, fma

ARITHS = ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw"]
QUASI = ("qdw", "qtw", "qqw")


class Ops:
    """The handful of operations CG needs, in one arithmetic; values are
    tuples of k floats (leading word first)."""

    def __init__(self, arith):
        self.arith = arith
        self.k = O.WORDS[arith]
        self.fp64 = arith == "fp64"

    def zero(self):
        return (0.0,) * self.k

    def promote(self, d):
        return (d,) + (0.0,) * (self.k - 1)

    def neg(self, a):
        return tuple(-w for w in a)

    def add(self, a, b):
        return (a[0] + b[0],) if self.fp64 else tuple(IMPL[self.arith]["add"](a, b))

    def mul(self, a, b):
        return (a[0] * b[0],) if self.fp64 else tuple(IMPL[self.arith]["mul"](a, b))

    def dxmul(self, d, a):
        return (d * a[0],) if self.fp64 else tuple(IMPL[self.arith]["dxmul"](d, a))

    def norm(self, a):
        return tuple(IMPL[self.arith]["norm"](a))

    def div(self, a, b):
        return (a[0] / b[0],) if self.fp64 else tuple(mw_div(self.arith, a, b))

    def to_fp64(self, a):
        if self.k == 1:
            return a[0]
        if self.k == 2:
            return a[0] + a[1]
        if self.k == 3:
            return a[0] + (a[1] + a[2])
        return a[0] + (a[1] + (a[2] + a[3]))

    # y + alpha * x with the FP64 solver's single fma
    def axpy(self, alpha, x, y):
        return (fma(alpha[0], x[0], y[0]),) if self.fp64 else self.add(y, self.mul(alpha, x))

    # y - alpha * x
    def axmy(self, alpha, x, y):
        return (fma(-alpha[0], x[0], y[0]),) if self.fp64 else self.add(y, self.neg(self.mul(alpha, x)))

    def spmv(self, A, v):
        out = []
        for i in range(A.n):
            acc = self.zero()
            for j in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
                a, x = float(A.val[j]), v[int(A.col_idx[j])]
                acc = (fma(a, x[0], acc[0]),) if self.fp64 else self.add(acc, self.dxmul(a, x))
            out.append(acc)
        return out

    def dot(self, u, v):
        acc = self.zero()
        for a, b in zip(u, v):
            acc = (fma(a[0], b[0], acc[0]),) if self.fp64 else self.add(acc, self.mul(a, b))
        return acc


def reading_cg(arith, A, b, x0, tol, maxit, normalise=1, jacobi=False, normalise_p=False):
    """CG (or Jacobi PCG) per Alg. 1 and the readings above.  Returns
    (x as k planes, iters, status, history)."""
    ops = Ops(arith)
    n = A.n
    x = [tuple(float(x0[w, i]) for w in range(ops.k)) for i in range(n)]
    d = None
    if jacobi:
        d = []
        for i in range(n):
            aii = 0.0
            for j in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
                if int(A.col_idx[j]) == i:
                    aii = float(A.val[j])
            d.append(1.0 / aii if aii != 0.0 else math.copysign(math.inf, aii))
    Ax = ops.spmv(A, x)
    if ops.fp64:
        r = [(float(b[i]) - Ax[i][0],) for i in range(n)]
    else:
        r = [ops.add(ops.promote(float(b[i])), ops.neg(Ax[i])) for i in range(n)]
    z = [ops.dxmul(d[i], r[i]) for i in range(n)] if jacobi else r
    p = list(z)
    rho = ops.dot(r, z)
    rr = ops.to_fp64(ops.dot(r, r)) if jacobi else ops.to_fp64(rho)
    bb = ops.dot([ops.promote(float(v)) for v in b], [ops.promote(float(v)) for v in b])
    nb = math.sqrt(ops.to_fp64(bb))
    hist = []
    planes = lambda v: np.array([[e[w] for e in v] for w in range(ops.k)])  # noqa: E731
    if rr == 0.0:
        return planes(x), 0, "ok", hist
    if maxit == 0:
        return planes(x), 0, "not_converged", hist
    it = 0
    while True:
        q = ops.spmv(A, p)
        sigma = ops.dot(p, q)
        s64 = ops.to_fp64(sigma)
        if not (s64 > 0.0) or not math.isfinite(s64):
            return planes(x), it, "breakdown", hist
        alpha = ops.div(rho, sigma)
        if not math.isfinite(ops.to_fp64(alpha)):
            return planes(x), it, "breakdown", hist
        x = [ops.axpy(alpha, p[i], x[i]) for i in range(n)]
        r = [ops.axmy(alpha, q[i], r[i]) for i in range(n)]
        if arith in QUASI and normalise > 0 and (it + 1) % normalise == 0:
            r = [ops.norm(v) for v in r]
            if normalise_p:
                p = [ops.norm(v) for v in p]
        if jacobi:
            z = [ops.dxmul(d[i], r[i]) for i in range(n)]
        else:
            z = r
        rho_new = ops.dot(r, z)
        rr = ops.to_fp64(ops.dot(r, r)) if jacobi else ops.to_fp64(rho_new)
        it += 1
        if not math.isfinite(rr) or not math.isfinite(ops.to_fp64(rho_new)):
            return planes(x), it, "breakdown", hist
        rel = math.sqrt(rr) / nb
        hist.append(rel)
        if rel < tol:
            return planes(x), it, "ok", hist
        if it >= maxit:
            return planes(x), it, "not_converged", hist
        beta = ops.div(rho_new, rho)
        p = [ops.axpy(beta, p[i], z[i]) for i in range(n)]
        rho = rho_new


def systems():
    """Small systems: 1D and 2D Poisson, a scaled banded SPD matrix (uneven
    diagonal, non-integer entries), a diagonal matrix with three distinct
    eigenvalues (stops with OK after 3 iterations), an indefinite one
    (breaks down)."""
    out = {}
    A = P.poisson1d(12)
    out["poisson1d"] = (A, P.uniform(A.n, 101))
    A = P.poisson2d(5)
    out["poisson2d"] = (A, P.uniform(A.n, 102))
    A = P.banded_spd(24, half_bw=3, seed=103, dseed=104)
    out["banded_scaled"] = (A, A.matvec(P.uniform(A.n, 105)))
    A = P.CSR.from_scipy(sp.diags(np.array([1.0, 2.0, 3.0] * 3)))
    out["diag3"] = (A, P.uniform(A.n, 106))
    M = P.poisson2d(4).to_scipy().tolil()
    M[0, 0] = -4.0
    out["indefinite"] = (P.CSR.from_scipy(M.tocsr()), np.eye(16)[0] + 0.25)
    return out


SYS = systems()


def compare(arith, A, b, x0=None, tol=1e-300, maxit=8, normalise=1, jacobi=False, normalise_p=False):
    k = O.WORDS[arith]
    x0 = np.zeros((k, A.n)) if x0 is None else x0
    xr, ir, sr, hr = reading_cg(arith, A, b, x0, tol, maxit, normalise, jacobi, normalise_p)
    xo, io = O.cg_solve(arith, A, b, x0=x0, tol=tol, maxit=maxit, normalise=normalise, history=True,
                        precond="jacobi" if jacobi else None, normalise_p=normalise_p)
    assert (io["iters"], io["status"]) == (ir, sr)
    assert np.array_equal(np.asarray(io["history"]).view(np.uint64), np.asarray(hr, dtype=np.float64).view(np.uint64))
    assert np.array_equal(xo.view(np.uint64), xr.view(np.uint64))
    return ir, sr


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("name", sorted(SYS))
def test_cg_reading_bit_exact(arith, name):
    A, b = SYS[name]
    # three distinct eigenvalues: exact CG stops after 3 steps (tol 1e-12)
    it, st = compare(arith, A, b, tol=1e-12 if name == "diag3" else 1e-300)
    want = {"diag3": ("ok", 3), "indefinite": ("breakdown", None)}.get(name, ("not_converged", 8))
    assert st == want[0] and (want[1] is None or it == want[1]), (st, it)


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_reading_from_nonzero_start(arith):
    """r0 = b - A x0 with a multi-word x0 (lower words nonzero)."""
    A, b = SYS["poisson2d"]
    k = O.WORDS[arith]
    rng = np.random.default_rng(107)
    x0 = np.stack([rng.uniform(-1, 1, A.n) * 2.0 ** (-54 * w) for w in range(k)])
    compare(arith, A, b, x0=x0)


@pytest.mark.parametrize("arith", QUASI)
@pytest.mark.parametrize("K", [0, 2, 3])
@pytest.mark.parametrize("name", ["poisson2d", "banded_scaled"])
def test_cg_reading_normalise_every_k(arith, K, name):
    A, b = SYS[name]
    compare(arith, A, b, normalise=K)


@pytest.mark.parametrize("arith", QUASI)
@pytest.mark.parametrize("K", [1, 2, 3])
@pytest.mark.parametrize("name", ["poisson2d", "banded_scaled"])
def test_cg_reading_normalise_r_and_p(arith, K, name):
    """The placement variant: p normalised with r, after its x update."""
    A, b = SYS[name]
    compare(arith, A, b, normalise=K, normalise_p=True)


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("name", ["poisson1d", "banded_scaled", "diag3"])
def test_pcg_reading_bit_exact(arith, name):
    A, b = SYS[name]
    it, st = compare(arith, A, b, jacobi=True, tol=1e-12 if name == "diag3" else 1e-300)
    if name == "diag3":
        # M^-1 A = I up to the rounding of 1 / a_ii: at most k steps
        assert st == "ok" and it <= O.WORDS[arith] + 1, (st, it)


@pytest.mark.parametrize("arith", ["fp64", "qtw"])
def test_cg_reading_stop_on_tolerance(arith):
    """A tolerance met inside the iteration budget: the stop iteration, the
    status and the residual history agree."""
    A, b = SYS["poisson2d"]
    it, st = compare(arith, A, b, tol=1e-4, maxit=25)
    assert st == "ok" and 1 < it < 25, (st, it)
