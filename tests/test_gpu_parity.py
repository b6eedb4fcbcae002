"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars:
  * element-wise ops and AXPY: bit-identical in every arithmetic (the
    paper's five and QTWE);
  * SpMV: bit-identical (both sum each row sequentially in CSR order);
  * DOT: within the format's bound against the exact dot:
    |d - x^T y| <= 2^-100 (2 words) / 2^-145 (3 words) * sum |x_i y_i|;
  * CG (plain, and Jacobi-preconditioned): same stopping criterion,
    iteration counts within 2 %, true residual (formed exactly by the
    oracle) within 10x of the oracle's.
"""
import zlib

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from conftest import rand_mw
from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu

ARITHS = ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw"]
DOT_BOUND = {1: 2.0 ** -45, 2: 2.0 ** -100, 3: 2.0 ** -145, 4: 2.0 ** -195}


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw as M
    M.lib()
    return M


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.cpu().numpy()


def special_values(k, n):
    """Word planes with zeros, signed zeros, powers of two, huge/tiny."""
    rng = np.random.default_rng(5)
    v = rand_mw(rng, k, n, emin=-300, emax=300)
    v[:, 0:8] = 0.0
    v[0, 1] = -0.0
    v[0, 2] = 1.0
    v[0, 3] = 2.0 ** -1000
    v[0, 4] = -2.0 ** 1000
    return v


# ------------------------------------------------------------ element-wise

@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("op", ["add", "mul", "dxmul", "div", "norm", "neg", "tofp64"])
@pytest.mark.parametrize("kind", ["normalised", "overlapping"])
def test_elementwise_bit_exact(mw, arith, op, kind):
    k = O.WORDS[arith]
    n = 3001  # several workgroups and a ragged tail
    rng = np.random.default_rng(zlib.crc32(("%s/%s/%s" % (arith, op, kind)).encode()))
    u = rand_mw(rng, k, n, normalised=(kind == "normalised"))
    v = rand_mw(rng, k, n, normalised=(kind == "normalised"))
    v[:, ::3] = -v[:, ::3]
    ua = u[0] if op == "dxmul" else u
    vv = v if op in ("add", "mul", "dxmul", "div") else None
    want = O.elementwise(arith, op, ua, vv)
    got = host(mw.elementwise(arith, op, dev(ua), dev(vv) if vv is not None else None))
    want = want.reshape(got.shape)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), \
        "first mismatch at %s" % (np.argwhere(got.view(np.uint64) != want.view(np.uint64))[:3],)


@pytest.mark.parametrize("arith", ARITHS)
def test_elementwise_special_values(mw, arith):
    k = O.WORDS[arith]
    u = special_values(k, 300)
    v = special_values(k, 300)[:, ::-1].copy()
    for op in ("add", "mul", "norm"):
        vv = v if op in ("add", "mul") else None
        want = O.elementwise(arith, op, u, vv)
        got = host(mw.elementwise(arith, op, dev(u), dev(vv) if vv is not None else None))
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), op


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("n", [1, 255, 256, 257, 70001])
def test_axpy_bit_exact(mw, arith, n):
    k = O.WORDS[arith]
    rng = np.random.default_rng(n)
    x = rand_mw(rng, k, n)
    y = rand_mw(rng, k, n)
    al = rand_mw(rng, k, 1)[:, 0]
    want = O.axpy(arith, al, x, y)
    yd = dev(y)
    mw.axpy(arith, dev(al), dev(x), yd)
    assert np.array_equal(host(yd).view(np.uint64), want.view(np.uint64))


# --------------------------------------------------------------------- SpMV

def ragged_matrix(seed=3):
    """Rows of very different lengths: empty rows, a row longer than one LDS
    chunk (3000 nonzeros), a dense-ish block; n not a multiple of 256."""
    rng = np.random.default_rng(seed)
    n = 5003
    rows, cols = [], []
    for i in range(n):
        if i % 97 == 5:
            continue  # empty row
        L = 3000 if i == 1234 else int(rng.integers(1, 40))
        c = np.unique(rng.integers(0, n, L))
        rows.append(np.full(c.size, i))
        cols.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = rng.standard_normal(r.size) * 10.0 ** rng.uniform(-3, 3, r.size)
    return P.CSR.from_scipy(sp.coo_matrix((v, (r, c)), shape=(n, n)))


def unsorted_matrix():
    # 3D Poisson rows with their CSR entries in a seeded random order: the
    # sum order is the stored order, which the plan must keep
    A = P.poisson3d(9, 8, 7)
    rng = np.random.default_rng(21)
    col, val = A.col_idx.copy(), A.val.copy()
    for i in range(A.n):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        perm = rng.permutation(b - a)
        col[a:b] = col[a:b][perm]
        val[a:b] = val[a:b][perm]
    return P.CSR(A.n, A.row_ptr.copy(), col, val)


def empty_slices_matrix():
    # 2D Poisson whose rows 64 .. 64 * 4 + 9 hold no entries at all: whole
    # empty slices (width 0) and a partly empty one between full ones
    A = P.poisson2d(30).to_scipy().tolil()
    for i in range(64, 64 * 4 + 10):
        A.rows[i] = []
        A.data[i] = []
    return P.CSR.from_scipy(A)


def reversed_matrix():
    # a circulant Laplacian with every row stored in descending column
    # order: slices away from the wrap-around still take diagonal slots, in
    # descending offset order
    A = P.circulant_laplacian(2500, [1, 3, 250], [0.5, 0.25, 1.0])
    col, val = A.col_idx.copy(), A.val.copy()
    for i in range(A.n):
        a, b = A.row_ptr[i], A.row_ptr[i + 1]
        col[a:b] = col[a:b][::-1]
        val[a:b] = val[a:b][::-1]
    return P.CSR(A.n, A.row_ptr.copy(), col, val)


def diagonal_slices(A):
    """Slices a SpMV plan stores as diagonal slots: slot j takes, from each
    of the 64 rows, its next CSR entry when that entry's column offset is the
    smallest among the rows' next entries; a slice qualifies when its rows
    are used up within its width (the longest row)."""
    ns = (A.n + 63) // 64
    count = 0
    for s in range(ns):
        rows = range(64 * s, min(64 * s + 64, A.n))
        offs = [list(A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]] - r) for r in rows]
        w = max(len(o) for o in offs)
        k = [0] * len(offs)
        for _ in range(w):
            cands = [o[kk] for o, kk in zip(offs, k) if kk < len(o)]
            if not cands:
                break
            m = min(cands)
            k = [kk + 1 if kk < len(o) and o[kk] == m else kk for o, kk in zip(offs, k)]
        if w > 0 and all(kk == len(o) for o, kk in zip(offs, k)):
            count += 1
    return count


MATRICES = {
    "poisson2d_64": lambda: P.poisson2d(64),
    "poisson3d_ragged": lambda: P.poisson3d(13, 11, 7),
    "banded27": lambda: P.banded_spd(5000, half_bw=13, seed=1, dseed=2),
    "circulant": lambda: P.circulant_laplacian(3001, [1, 17, 400, 1200], [0.5, 0.3, 1.0, 0.2]),
    "ragged": ragged_matrix,
    "unsorted": unsorted_matrix,
    "reversed": reversed_matrix,
    "empty_slices": empty_slices_matrix,
}


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("mat", list(MATRICES))
def test_spmv_bit_exact(mw, arith, mat):
    A = MATRICES[mat]()
    k = O.WORDS[arith]
    x = rand_mw(np.random.default_rng(11), k, A.n, emin=-4, emax=4)
    want = O.spmv(arith, A, x)
    Ad = mw.DeviceCSR.from_host(A)
    got = host(mw.spmv(arith, Ad, dev(x)))
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("arith", ARITHS)
def test_spmv_integer_exact(mw, arith):
    A = P.poisson3d(17, 9, 6)
    x = P.integer_vector(A.n, seed=2)
    got = host(mw.spmv(arith, mw.DeviceCSR.from_host(A), dev(x.reshape(1, -1).repeat(O.WORDS[arith], 0) *
                                                              np.array([[1.0]] + [[0.0]] * (O.WORDS[arith] - 1)))))
    ref = (A.to_scipy().astype(np.int64) @ x.astype(np.int64)).astype(np.float64)
    assert np.array_equal(got[0], ref) and np.all(got[1:] == 0.0)


# ---------------------------------------------------------------------- DOT

@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("n", [1, 255, 2048, 2049, 100003, 2 ** 21, 2 ** 21 + 5])
def test_dot_within_bound(mw, arith, n):
    k = O.WORDS[arith]
    rng = np.random.default_rng(n + 7)
    x = rand_mw(rng, k, n, emin=-6, emax=6)
    y = rand_mw(rng, k, n, emin=-6, emax=6)
    d = host(mw.dot(arith, dev(x), dev(y)))
    err, sc = O.dot_error(arith, x, y, d)
    assert err <= DOT_BOUND[k] * sc, (err / sc)
    d2 = host(mw.dot(arith, dev(x), dev(y)))
    assert np.array_equal(d, d2)  # run-to-run reproducible


def test_dot_empty(mw):
    import torch
    for arith in ARITHS:
        k = O.WORDS[arith]
        z = torch.empty((k, 0), dtype=torch.float64, device="cuda")
        assert np.all(host(mw.dot(arith, z, z)) == 0.0)


# ----------------------------------------------------------------------- CG

def cg_parity(mw, arith, A, b, tol, maxit=None, precond=None):
    xo, io = O.cg_solve(arith, A, b, tol=tol, maxit=maxit, precond=precond)
    Ad = mw.DeviceCSR.from_host(A)
    xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=tol, maxit=maxit, precond=precond)
    xg = host(xg)
    assert ig["status"] == io["status"], (ig, io)
    assert abs(ig["iters"] - io["iters"]) <= max(1, int(0.02 * io["iters"])), (ig["iters"], io["iters"])
    tro = O.true_residual(arith, A, b, xo)
    trg = O.true_residual(arith, A, b, xg)
    nb = np.linalg.norm(b)
    floor = 1e-300
    assert trg / nb <= 10 * max(tro / nb, floor), (trg / nb, tro / nb)
    return xg, ig, io


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_poisson2d_64(mw, arith):
    A, b, _ = P.case_poisson2d_64()
    cg_parity(mw, arith, A, b, 1e-12)


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_poisson3d_small(mw, arith):
    A, b, _ = P.case_poisson3d(nx=24)
    cg_parity(mw, arith, A, b, 1e-12)


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_initial_guess(mw, arith):
    """A nonzero x0 (random multi-word planes): r0 = b - A x0 on both sides."""
    A, b, _ = P.case_poisson3d(nx=16)
    k = O.WORDS[arith]
    x0 = rand_mw(np.random.default_rng(17), k, A.n, emin=-2, emax=2)
    xo, io = O.cg_solve(arith, A, b, x0=x0, tol=1e-12)
    xg, ig = mw.cg_solve(arith, mw.DeviceCSR.from_host(A), dev(b), x=dev(x0), tol=1e-12)
    assert ig["status"] == io["status"] == "ok"
    assert abs(ig["iters"] - io["iters"]) <= max(1, int(0.02 * io["iters"]))
    tro = O.true_residual(arith, A, b, xo)
    trg = O.true_residual(arith, A, b, host(xg))
    assert trg <= 10 * tro, (trg, tro)


@pytest.mark.parametrize("n", [1, 5, 65, 64 * 16 + 1])
def test_cg_tiny_and_ragged_sizes(mw, n):
    """Systems smaller than one slice or tile, and one row past a boundary."""
    A = P.poisson1d(n)
    b = A.matvec(np.random.default_rng(n).uniform(-1, 1, n))
    for arith in ("fp64", "qtw"):
        cg_parity(mw, arith, A, b, 1e-12)


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_tight_tolerance(mw, arith):
    """Manufactured integer solution (b = A x* exact): at a tolerance near
    each arithmetic's resolution the error against x* is about ten times the
    tolerance (the oracle's: 1.2e-13, 7.1e-28, 4.2e-40)."""
    A = P.poisson2d(40, 30)
    xs = P.integer_vector(A.n, seed=3)
    b = A.matvec(xs)
    tol = {"fp64": 1e-14, "dw": 1e-28, "qdw": 1e-28, "tw": 1e-40, "qtw": 1e-40, "qtwe": 1e-40,
           "qw": 1e-55, "qqw": 1e-55}[arith]
    xg, ig, io = cg_parity(mw, arith, A, b, tol)
    # x_0 - x* is exact (x_0 is within a few units in the last place of the
    # integer); the lower words are then small enough to add in FP64
    e = xg[0] - xs
    for w in range(1, xg.shape[0]):
        e = e + xg[w]
    err = np.abs(e).max() / np.abs(xs).max()
    assert err < {"fp64": 1e-12, "dw": 1e-26, "qdw": 1e-26, "tw": 1e-38, "qtw": 1e-38, "qtwe": 1e-38,
                  "qw": 1e-53, "qqw": 1e-53}[arith]


def _diag_indefinite(seed, n=24):
    """A diagonal with one to three negative entries and a random b; the
    seeds used below break down (p^T q <= 0) after 1, 2, 3, 4 and 5
    completed iterations."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 4.0, n)
    neg = rng.integers(1, 4)
    d[rng.choice(n, neg, replace=False)] *= -rng.uniform(0.05, 1.0, neg)
    return P.CSR.from_scipy(sp.diags(d, 0).tocsr()), rng.uniform(-1, 1, n)


def _x_close(arith, xg, xo):
    """Largest |x_gpu - x_oracle| / max|x_oracle|, the words' differences
    added up (the leading words agree closely, so the sum is accurate)."""
    e = np.zeros(xo.shape[1])
    for w in range(xo.shape[0]):
        e = e + (xg[w] - xo[w])
    return np.abs(e).max() / np.abs(xo[0]).max()


X_BOUND = {"fp64": 1e-13, "dw": 1e-26, "qdw": 1e-26, "tw": 1e-38, "qtw": 1e-38, "qtwe": 1e-38,
           "qw": 1e-53, "qqw": 1e-53}


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_x_after_each_stop_position(mw, arith):
    """x at every stop position: after m = 1..6 iterations (maxit = m) and
    after a breakdown following 1..5 iterations.  The solver applies the
    x updates of two iterations in one pass for 3-word types, so these are
    the stops at both positions of a pair, with and without a pending
    update.  x equals the oracle's up to the rounding of the dots."""
    A, b, _ = P.case_poisson3d(nx=12)
    Ad = mw.DeviceCSR.from_host(A)
    for m in range(1, 7):
        xo, io = O.cg_solve(arith, A, b, tol=0.0, maxit=m)
        xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=0.0, maxit=m)
        assert ig["status"] == io["status"] == "not_converged" and ig["iters"] == io["iters"] == m
        assert _x_close(arith, host(xg), np.asarray(xo).reshape(-1, A.n)) < X_BOUND[arith], m
    for seed, iters in ((3, 1), (1, 2), (0, 3), (64, 4), (191, 5)):
        M, bm = _diag_indefinite(seed)
        xo, io = O.cg_solve(arith, M, bm, tol=1e-14)
        xg, ig = mw.cg_solve(arith, mw.DeviceCSR.from_host(M), dev(bm), tol=1e-14)
        assert io["status"] == ig["status"] == "breakdown", (seed, io, ig)
        assert io["iters"] == ig["iters"] == iters, (seed, io, ig)
        assert _x_close(arith, host(xg), np.asarray(xo).reshape(-1, M.n)) < X_BOUND[arith], seed


# ------------------------------------------ vector-row SpMV plans (CSRVEC)

def _wide_matrix(seed=21, n=3001):
    """Rows of 0..600 entries (empty rows, long rows, random columns), n not
    a multiple of any rows-per-tile count."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 600, n)
    lens[::97] = 0
    rows, cols = [], []
    for i, ln in enumerate(lens):
        c = np.unique(rng.integers(0, n, ln))
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    vals = rng.standard_normal(rows.size) * 2.0 ** rng.integers(-8, 8, rows.size)
    return P.CSR.from_scipy(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)))


VEC_MATRICES = {
    "wide_random": _wide_matrix,
    "banded_150": lambda: P.banded_spd(2000, half_bw=150, seed=5, scale=False),
    "poisson3d": lambda: P.poisson3d(17, 9, 6),
}


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("mat", list(VEC_MATRICES))
@pytest.mark.parametrize("lanes", [2, 8, 64])
def test_spmv_rows_within_bound(mw, arith, mat, lanes):
    """Vector-row plan: each row's sum is associated differently from CSR
    order, so it is checked against the exact row sum: |y_i - (Ax)_i| <=
    8 (path + 2) u^k sum_j |a_ij x_j|, path = ceil(len / L) + log2 L
    (u = 2^-53); and reproducible run to run."""
    A = VEC_MATRICES[mat]()
    k = O.WORDS[arith]
    x = rand_mw(np.random.default_rng(31), k, A.n, emin=-4, emax=4)
    Ad = mw.DeviceCSR.from_host(A)
    plan = mw.Plan(Ad, rows=lanes)
    assert plan.format == "csrvec" and plan.lanes == lanes
    y1 = host(mw.spmv_planned(arith, plan, dev(x)))
    y2 = host(mw.spmv_planned(arith, plan, dev(x)))
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    err, sc = O.spmv_error(arith, A, x, y1)
    lens = np.diff(A.row_ptr)
    path = np.ceil(lens / lanes) + np.log2(lanes)
    bound = 8 * (path + 2) * 2.0 ** (-53 * k) * sc
    assert np.all(err <= bound), np.max(err / np.maximum(bound, 1e-300))
    empty = lens == 0
    assert np.all(y1[:, empty] == 0.0)


@pytest.mark.parametrize("arith", ARITHS)
def test_spmv_rows_tiny_and_ragged(mw, arith):
    """Vector-row plans at n = 1, 2, 63, 65, 257 (a single tile, a ragged
    last tile) and one row longer than 64 x L entries, every L: within the
    row-sum bound, and the CG on a tiny SPD system with a vector plan agrees
    with the oracle."""
    k = O.WORDS[arith]
    rng = np.random.default_rng(17)
    mats = []
    for n in (1, 2, 63, 65, 257):
        M = sp.random(n, n, density=min(1.0, 9.0 / n), random_state=rng, format="csr") + sp.eye(n)
        mats.append(P.CSR.from_scipy(M))
    long_row = sp.lil_matrix((5000, 5000))
    long_row[5, :] = rng.standard_normal(5000)               # 5000 > 64 x 64 entries in one row
    mats.append(P.CSR.from_scipy(long_row.tocsr() + sp.eye(5000)))
    for A in mats:
        x = rand_mw(np.random.default_rng(A.n), k, A.n, emin=-3, emax=3)
        Ad = mw.DeviceCSR.from_host(A)
        for lanes in (2, 4, 8, 16, 32, 64):
            y = host(mw.spmv_planned(arith, mw.Plan(Ad, rows=lanes), dev(x)))
            err, sc = O.spmv_error(arith, A, x, y)
            lens = np.diff(A.row_ptr)
            bound = 8 * (np.ceil(lens / lanes) + np.log2(lanes) + 2) * 2.0 ** (-53 * k) * sc
            assert np.all(err <= bound), (A.n, lanes)
    A = P.poisson2d(3, 2)
    b = A.matvec(np.arange(1.0, A.n + 1))
    Ad = mw.DeviceCSR.from_host(A)
    xo, io = O.cg_solve(arith, A, b, tol=1e-12)
    for lanes in (2, 64):
        xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, plan=mw.Plan(Ad, rows=lanes))
        assert ig["status"] == io["status"] == "ok" and abs(ig["iters"] - io["iters"]) <= 1


def _normal_matrix(seed=9, n=3000, k=6, shift=0.01):
    """B^T B + shift I, B random sparse (k entries per row on average): SPD,
    rows of 1 to ~100 entries (about 37 on average), ~400 CG iterations."""
    B = sp.random(n, n, density=k / n, random_state=np.random.default_rng(seed), format="csr")
    return P.CSR.from_scipy((B.T @ B + shift * sp.eye(n)).tocsr())


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_with_vector_row_plans(mw, arith):
    """CG on a matrix with long rows: with the plan the solver picks itself
    for such a matrix (average row length >= 32, n <= 2^18: vector rows) and
    with explicit vector-row plans.  The row sums are associated differently
    from the oracle's CSR order; the iteration counts stay within the 2 %
    bar (measured over six seeds of this matrix: FP64 0.3-0.8 %, DW
    0-0.5 %)."""
    A = _normal_matrix()
    b = A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n))
    xo, io = O.cg_solve(arith, A, b, tol=1e-12)
    nb = np.linalg.norm(b)
    tro = O.true_residual(arith, A, b, xo) / nb
    Ad = mw.DeviceCSR.from_host(A)
    slack = 0.02
    for lanes in (None, 4, 32):
        plan = None if lanes is None else mw.Plan(Ad, rows=lanes)
        xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, plan=plan)
        assert ig["status"] == io["status"] == "ok", (lanes, ig, io)
        assert abs(ig["iters"] - io["iters"]) <= max(1, int(slack * io["iters"])), (lanes, ig["iters"], io["iters"])
        assert O.true_residual(arith, A, b, host(xg)) / nb <= 10 * tro, lanes


def _irregular_spd(n=20000, seed=4):
    """Symmetric, strictly diagonally dominant, rows of 2 .. 2269 entries
    (23.5 on average): SELL-64 would store 2.3x the entries, so a plan falls
    back to CSR and the solver takes vector rows instead."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 25, n)
    rows = np.repeat(np.arange(n), lens)
    cols = np.clip(rows + rng.integers(-3000, 3001, rows.size), 0, n - 1)
    S = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n))
    M = (S + S.T).tocsr()
    M.setdiag(0)
    M.eliminate_zeros()
    d = np.asarray(abs(M).sum(axis=1)).ravel() + 1.0
    return P.CSR.from_scipy((M + sp.diags(d)).tocsr())


@pytest.mark.parametrize("arith", ARITHS)
def test_solver_plan_choice_and_irregular_rows(mw, arith):
    """mw_cg_plan gives the plan the solver builds for itself: SELL-64 for a
    Poisson matrix, vector rows by size for few long rows, vector rows for
    irregular rows (SELL's CSR fallback).  On the irregular matrix the
    solver's own choice keeps the parity bar, and passing that plan
    explicitly gives the same bits."""
    lanes_by_size = 8 if arith == "fp64" else 4      # ~37 entries per row
    lanes_irregular = 4 if arith == "fp64" else 2    # ~23.5 entries per row
    assert mw.Plan(mw.DeviceCSR.from_host(P.poisson3d(20)), solver=arith).format == "sell64"
    pw = mw.Plan(mw.DeviceCSR.from_host(_normal_matrix()), solver=arith)
    assert (pw.format, pw.lanes) == ("csrvec", lanes_by_size)
    A = _irregular_spd()
    Ad = mw.DeviceCSR.from_host(A)
    assert mw.Plan(Ad).format == "csr"
    pl = mw.Plan(Ad, solver=arith)
    assert (pl.format, pl.lanes) == ("csrvec", lanes_irregular)
    b = A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n))
    xo, io = O.cg_solve(arith, A, b, tol=1e-12)
    x1, i1 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12)
    x2, i2 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, plan=pl)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1).view(np.uint64), host(x2).view(np.uint64))
    assert i1["status"] == io["status"] == "ok"
    # FP64 on this matrix: 84 iterations against the oracle's 87.  Its rows
    # of up to 2269 entries, summed by lane trees, round less than the
    # oracle's sequential sums, and FP64 CG here moves toward the count of
    # nearly exact arithmetic (DW: 75 iterations); moving five entries of b
    # by one ulp changes the oracle's own FP64 count by one.  The 2 % bar
    # holds for every multi-word arithmetic.
    slack = 0.04 if arith == "fp64" else 0.02
    assert abs(i1["iters"] - io["iters"]) <= max(1, int(slack * io["iters"])), (i1["iters"], io["iters"])
    nb = np.linalg.norm(b)
    assert O.true_residual(arith, A, b, host(x1)) / nb <= 10 * O.true_residual(arith, A, b, xo) / nb


# ------------------------------------- Jacobi-preconditioned CG (extension)

def _shifted_laplacian(seed=12):
    """2D Laplacian with a random diagonal shift: a non-constant diagonal."""
    A = P.poisson2d(30, 27).to_scipy().tolil()
    rng = np.random.default_rng(seed)
    for i in range(A.shape[0]):
        A[i, i] = A[i, i] + rng.uniform(0.0, 3.0)
    A = P.CSR.from_scipy(A.tocsr())
    return A, A.matvec(rng.uniform(-1, 1, A.n))


PCG_CASES = {
    "banded_scaled": lambda: P.case_banded_illcond(n=2048)[:2],
    "poisson3d_16": lambda: P.case_poisson3d(nx=16)[:2],
    "shifted_laplacian": _shifted_laplacian,
}


@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("case", list(PCG_CASES))
def test_pcg_jacobi_parity(mw, arith, case):
    A, b = PCG_CASES[case]()
    xg, ig, io = cg_parity(mw, arith, A, b, 1e-10, maxit=3000, precond="jacobi")
    assert ig["status"] == "ok"


@pytest.mark.parametrize("arith", ARITHS)
def test_pcg_jacobi_diagonal_four_is_cg(mw, arith):
    """Diagonal 4: M^-1 = I/4 is exact and PCG is CG scaled by powers of two
    throughout, so on the GPU too it reproduces the plain solve bit for bit."""
    A, b, _ = P.case_poisson2d_64()
    Ad = mw.DeviceCSR.from_host(A)
    x1, i1 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12)
    x2, i2 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, precond="jacobi")
    assert i1["iters"] == i2["iters"] and i1["rel_res"] == i2["rel_res"]
    assert np.array_equal(host(x1).view(np.uint64), host(x2).view(np.uint64))


@pytest.mark.parametrize("arith", ARITHS)
def test_pcg_jacobi_stop_positions_and_breakdown(mw, arith):
    A, b = _shifted_laplacian(seed=13)
    Ad = mw.DeviceCSR.from_host(A)
    for m in range(1, 7):
        xo, io = O.cg_solve(arith, A, b, tol=0.0, maxit=m, precond="jacobi")
        xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=0.0, maxit=m, precond="jacobi")
        assert ig["status"] == io["status"] == "not_converged" and ig["iters"] == io["iters"] == m
        assert _x_close(arith, host(xg), np.asarray(xo).reshape(-1, A.n)) < X_BOUND[arith], m
    M = P.CSR.from_scipy(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]])))
    _, info = mw.cg_solve(arith, mw.DeviceCSR.from_host(M), dev(np.array([1.0, 1.0])), precond="jacobi")
    assert info["status"] == "breakdown" and info["iters"] == 0
    with pytest.raises(mw.MWError):
        mw.cg_solve(arith, Ad, dev(b), precond="ilu")


@pytest.mark.parametrize("arith", ARITHS)
def test_cg_failure_paths(mw, arith):
    A, b, _ = P.case_poisson2d_64()
    Ad = mw.DeviceCSR.from_host(A)
    _, i = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, maxit=7)
    assert i["status"] == "not_converged" and i["iters"] == 7
    _, i = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, maxit=0)
    assert i["status"] == "not_converged" and i["iters"] == 0
    x, i = mw.cg_solve(arith, Ad, dev(np.zeros(A.n)), tol=1e-12)
    assert i["status"] == "ok" and i["iters"] == 0 and not host(x).any()
    M2 = P.CSR.from_scipy(sp.diags(np.array([-1.0] + [1.0] * 9), 0))
    e0 = np.zeros(10)
    e0[0] = 1.0
    _, i = mw.cg_solve(arith, mw.DeviceCSR.from_host(M2), dev(e0), tol=1e-12)
    assert i["status"] == "breakdown" and i["iters"] == 0


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_cg_deterministic(mw, arith):
    A, b, _ = P.case_poisson3d(nx=20)
    Ad = mw.DeviceCSR.from_host(A)
    x1, i1 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12)
    x2, i2 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1).view(np.uint64), host(x2).view(np.uint64))


def test_cg_graph_cache_alternating_configurations(mw):
    """Ten solve configurations (arithmetic x matrix x preconditioner), more
    than the per-thread cache of captured chunks holds, cycled twice: every
    solve equals the same solve with direct launches, bit for bit, whether
    its graph was reused, evicted or captured again."""
    mats = [P.case_poisson3d(nx=14)[:2], P.case_poisson2d_64()[:2]]
    devs = [(mw.DeviceCSR.from_host(A), dev(b)) for A, b in mats]
    configs = [(ar, m, pc) for m in range(2) for ar in ("fp64", "dw", "qtw", "tw", "qtwe") for pc in (None,)]
    configs = configs[:8] + [("dw", 0, "jacobi"), ("qtw", 1, "jacobi")]
    import torch
    ref, bufs = {}, {}
    for cfg in configs:
        ar, m, pc = cfg
        Ad, bd = devs[m]
        # one workspace and one x per configuration: the graph key holds their addresses
        bufs[cfg] = (mw.cg_workspace(ar, Ad), torch.zeros((mw.WORDS[ar], Ad.n), dtype=torch.float64, device="cuda"))
        x, _ = mw.cg_solve(ar, Ad, bd, tol=1e-12, precond=pc, graph=False, chunk=8)
        ref[cfg] = host(x)
    for _ in range(2):
        for cfg in configs:
            ar, m, pc = cfg
            ws, x = bufs[cfg]
            x.zero_()
            _, info = mw.cg_solve(ar, devs[m][0], devs[m][1], x=x, tol=1e-12, precond=pc, chunk=8, workspace=ws)
            assert info["status"] == "ok"
            assert np.array_equal(host(x).view(np.uint64), ref[cfg].view(np.uint64)), cfg


def test_cg_history_and_nn(mw):
    A = P.poisson2d(24, 20)
    b = A.matvec(P.integer_vector(A.n, seed=3))
    Ad = mw.DeviceCSR.from_host(A)
    _, i = mw.cg_solve("qtw", Ad, dev(b), tol=1e-30, history=True)
    h = i["history"]
    assert h.size == i["iters"] and h[-1] < 1e-30 and h[0] > 1e-30
    # without normalisation the quasi variants fail to converge (Sec. V-B)
    _, nn = mw.cg_solve("qdw", Ad, dev(b), tol=1e-28, maxit=4000, normalize=False)
    _, on = O.cg_solve("qdw", A, b, tol=1e-28, maxit=4000, normalise=False)
    assert nn["status"] != "ok" and on["status"] != "ok"


@pytest.mark.parametrize("arith", ["qdw", "qtw"])
def test_cg_normalisation_frequency(mw, arith):
    """normalize = K (r normalised in iterations K, 2K, ...): the GPU takes
    the same iterations as the oracle.  C1 at K = 2 breaks down near
    iteration 75 in both, so 60 iterations are compared (tol = 0): same
    status and count, true residual within 10x of the oracle's; plus the
    bitwise consequences of the schedule on the GPU itself."""
    A, b, _ = P.case_poisson2d_64()
    Ad = mw.DeviceCSR.from_host(A)
    bd = dev(b)
    xo, io = O.cg_solve(arith, A, b, tol=0.0, maxit=60, normalise=2)
    xg, ig = mw.cg_solve(arith, Ad, bd, tol=0.0, maxit=60, normalize=2)
    assert ig["status"] == io["status"] == "not_converged" and ig["iters"] == io["iters"] == 60
    tro = O.true_residual(arith, A, b, xo)
    trg = O.true_residual(arith, A, b, host(xg))
    assert trg <= 10 * tro, (trg, tro)
    one2, _ = mw.cg_solve(arith, Ad, bd, tol=0.0, maxit=1, normalize=2)
    one0, _ = mw.cg_solve(arith, Ad, bd, tol=0.0, maxit=1, normalize=0)
    assert np.array_equal(host(one2).view(np.uint64), host(one0).view(np.uint64))
    three2, _ = mw.cg_solve(arith, Ad, bd, tol=0.0, maxit=3, normalize=2)
    three0, _ = mw.cg_solve(arith, Ad, bd, tol=0.0, maxit=3, normalize=0)
    assert not np.array_equal(host(three2).view(np.uint64), host(three0).view(np.uint64))
    big, ib = mw.cg_solve(arith, Ad, bd, tol=1e-12, maxit=300, normalize=10 ** 6)
    nn, inn = mw.cg_solve(arith, Ad, bd, tol=1e-12, maxit=300, normalize=0)
    assert ib["iters"] == inn["iters"] and np.array_equal(host(big).view(np.uint64), host(nn).view(np.uint64))
    with pytest.raises(mw.MWError):
        mw.cg_solve(arith, Ad, bd, normalize=-1)


@pytest.mark.parametrize("arith", ["qdw", "qtw", "qqw"])
@pytest.mark.parametrize("K", [2, 8])
def test_cg_normalise_r_and_p(mw, arith, K):
    """The placement variant normalize_p (p normalised with r in iterations
    K, 2K, ...): on C1 it converges where normalising r alone breaks down.
    Against the oracle's variant: same status, iterations within 2 %, true
    residual within 10x; graph replay and direct launches give the same
    bits; with a preconditioner it is rejected."""
    A, b, _ = P.case_poisson2d_64()
    Ad = mw.DeviceCSR.from_host(A)
    xo, io = O.cg_solve(arith, A, b, tol=1e-12, normalise=K, normalise_p=True)
    xg, ig = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, normalize=K, normalize_p=True)
    assert ig["status"] == io["status"] == "ok"
    assert abs(ig["iters"] - io["iters"]) <= max(1, int(0.02 * io["iters"])), (ig, io)
    tro = O.true_residual(arith, A, b, xo)
    assert O.true_residual(arith, A, b, host(xg)) <= 10 * tro
    xd, idd = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, normalize=K, normalize_p=True, graph=False)
    assert idd["iters"] == ig["iters"] and np.array_equal(host(xd).view(np.uint64), host(xg).view(np.uint64))
    with pytest.raises(mw.MWError):
        mw.cg_solve(arith, Ad, dev(b), normalize=K, normalize_p=True, precond="jacobi")


# ----------------------------------------------------------- planned SpMV

@pytest.mark.parametrize("arith", ARITHS)
@pytest.mark.parametrize("mat", list(MATRICES))
def test_spmv_planned_bit_exact(mw, arith, mat):
    A = MATRICES[mat]()
    k = O.WORDS[arith]
    x = rand_mw(np.random.default_rng(12), k, A.n, emin=-4, emax=4)
    want = O.spmv(arith, A, x)
    plan = mw.Plan(mw.DeviceCSR.from_host(A))
    # a row far longer than its slice-mates makes the padding too large:
    # the plan falls back to the CSR kernel
    assert plan.format == ("csr" if mat == "ragged" else "sell64")
    if plan.format == "sell64":
        assert plan.stored >= A.nnz and plan.stored % 64 == 0
        # stencil / banded slices become diagonal slots, the circulant's
        # wrap-around slices and the shuffled rows keep explicit columns
        assert plan.ndiag == diagonal_slices(A)
        ns = (A.n + 63) // 64
        if mat in ("poisson2d_64", "banded27"):
            assert plan.ndiag == ns
        if mat == "circulant":
            assert 0 < plan.ndiag < ns
    got = host(mw.spmv_planned(arith, plan, dev(x)))
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_spmv_planned_tiny_and_ragged_tail(mw):
    # n smaller than one slice, and n one past a slice boundary
    for n in (1, 5, 65, 64 * 8 + 1):
        A = P.poisson1d(n)
        for arith in ("fp64", "qtw"):
            x = rand_mw(np.random.default_rng(n), O.WORDS[arith], n)
            want = O.spmv(arith, A, x)
            plan = mw.Plan(mw.DeviceCSR.from_host(A))
            got = host(mw.spmv_planned(arith, plan, dev(x)))
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (n, arith)


# --------------------------------------------- graphs, plans and timing

@pytest.mark.parametrize("arith", ["fp64", "qtw"])
def test_cg_graph_replays_match_direct_launches(mw, arith):
    import torch
    A, b, _ = P.case_poisson3d(nx=20)
    Ad = mw.DeviceCSR.from_host(A)
    bd = dev(b)
    ws = mw.cg_workspace(arith, Ad)
    k = O.WORDS[arith]
    x = torch.zeros((k, A.n), dtype=torch.float64, device="cuda")
    _, ref = mw.cg_solve(arith, Ad, bd, x=x, tol=1e-12, workspace=ws, graph=False)
    xref = host(x).copy()
    for rep in range(3):  # the captured chunk is reused by every solve
        x.zero_()
        junk = torch.ones(1000, device="cuda").cumsum(0)  # eager work between replays
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=1e-12, workspace=ws, chunk=8)
        assert junk[-1].item() == 1000.0
        assert info["iters"] == ref["iters"] and info["status"] == "ok"
        assert np.array_equal(host(x).view(np.uint64), xref.view(np.uint64)), rep


def test_cg_with_plan_and_timing(mw):
    A, b, _ = P.case_poisson3d(nx=24)
    Ad = mw.DeviceCSR.from_host(A)
    plan = mw.Plan(Ad)
    x1, i1 = mw.cg_solve("dw", Ad, dev(b), tol=1e-12)
    prof = mw.CgProf.of("spmv")
    x2, i2 = mw.cg_solve("dw", Ad, dev(b), tol=1e-12, plan=plan, prof=prof)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1).view(np.uint64), host(x2).view(np.uint64))
    d = prof.as_dict()
    assert d["spmv"]["launches"] == i2["iters"] - 1 and d["spmv"]["ms"] > 0
    assert d["update_r"]["launches"] == 0


@pytest.mark.parametrize("arith", ["fp64", "dw", "qtw", "qqw"])
def test_cg_bits_do_not_depend_on_chunk_length(mw, arith):
    """Iterations per captured graph (1 and 5, rounded up to even, 32, 100)
    change only where the host polls the stop flag: x and the iteration
    count are bit-identical, also when the stop falls inside a chunk."""
    A = P.poisson3d(20, 18, 16)
    b = A.matvec(np.random.default_rng(31).uniform(-1.0, 1.0, A.n))
    Ad = mw.DeviceCSR.from_host(A)
    runs = [mw.cg_solve(arith, Ad, dev(b), tol=1e-12, chunk=c) for c in (1, 5, 32, 100)]
    x0, i0 = runs[0]
    assert i0["status"] == "ok" and i0["iters"] % 100 != 0   # the stop inside a chunk of 100
    for x, info in runs[1:]:
        assert info["iters"] == i0["iters"] and info["status"] == i0["status"]
        assert np.array_equal(x.cpu().numpy().view(np.uint64), x0.cpu().numpy().view(np.uint64))
