"""Batched CG (many independent systems in one lockstep solve) on the GPU,
against the CPU oracle run system by system and against the single-system
GPU solver.  Bars as for CG: same status, iterations within 2 %, true
residual within 10x of the oracle's."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from conftest import rand_mw
from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def small_batch():
    """20 uneven systems (Poisson 2D/3D, circulant) plus: a zero right-hand
    side, a single-row system, and an indefinite system (breaks down)."""
    B = P.batch_systems(nsys=20, seed=11, nmin=100, nmax=3000)
    mats = [B.system(s)[0] for s in range(B.nsys)]
    bs = [B.system(s)[1] for s in range(B.nsys)]
    bs[3] = np.zeros_like(bs[3])
    mats.append(P.CSR.from_scipy(sp.identity(1) * 2.0))
    bs.append(np.array([3.0]))
    M = P.poisson2d(12).to_scipy().tolil()
    M[0, 0] = -4.0
    mats.append(P.CSR.from_scipy(M))
    e0 = np.zeros(144)
    e0[0] = 1.0
    bs.append(e0)
    return mats, bs, P.batch_from_systems(mats, bs)


# the mixed types (FP64 vectors, SpMV rows and dots in DW / QTW) against the
# oracle's mixed solve in their base arithmetic
MIXED = {"mxdw": "dw", "mxqtw": "qtw"}


@pytest.mark.parametrize("arith", ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw", "mxdw", "mxqtw"])
def test_batched_matches_oracle_per_system(mw, small_batch, arith):
    mats, bs, B = small_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    x, iters, status, rel, info = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=20000)
    x = x.cpu().numpy()
    assert x.shape[0] == mw.WORDS[arith]
    off = B.sys_row_off
    va = "fp64" if arith in MIXED else arith  # the arithmetic of the stored x
    for s, (A, b) in enumerate(zip(mats, bs)):
        if arith in MIXED:
            xo, io = O.cg_solve(MIXED[arith], A, b, tol=1e-12, maxit=20000, mixed=True)
        else:
            xo, io = O.cg_solve(arith, A, b, tol=1e-12, maxit=20000)
        st = {0: "ok", 1: "not_converged", 2: "breakdown"}[int(status[s])]
        assert st == io["status"], (s, st, io)
        assert abs(int(iters[s]) - io["iters"]) <= max(1, int(0.02 * io["iters"])), (s, iters[s], io["iters"])
        if io["status"] == "ok" and np.any(b):
            xs = x[:, off[s]:off[s + 1]]
            nb = np.linalg.norm(b)
            trg = O.true_residual(va, A, b, xs) / nb
            tro = O.true_residual(va, A, b, xo) / nb
            assert trg <= 10 * max(tro, 1e-300), (s, trg, tro)
    assert int(iters[3]) == 0 and int(status[3]) == 0          # b = 0
    assert int(status[-1]) == 2                                 # indefinite system
    assert info["status"] == "breakdown"


def test_batched_matches_single_solver_and_is_deterministic(mw, small_batch):
    mats, bs, B = small_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    x1, it1, st1, _, _ = mw.cg_solve_batched("qtw", Ad, B.sys_row_off, dev(B.b), tol=1e-12)
    x2, it2, st2, _, _ = mw.cg_solve_batched("qtw", Ad, B.sys_row_off, dev(B.b), tol=1e-12, graph=False)
    assert np.array_equal(it1, it2) and np.array_equal(st1, st2)
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))
    for s in range(0, len(mats), 4):
        _, i = mw.cg_solve("qtw", mw.DeviceCSR.from_host(mats[s]), dev(bs[s]), tol=1e-12)
        assert abs(i["iters"] - int(it1[s])) <= max(1, int(0.02 * i["iters"])), (s, i, it1[s])


@pytest.mark.parametrize("arith", ["fp64", "qtw", "mxdw"])
def test_batched_empty_systems(mw, small_batch, arith):
    """Systems of zero rows (repeated row offsets) at the start, inside and
    at the end of the batch: each stops at once (status ok, 0 iterations,
    relative residual 0), and every other system's x, iterations and status
    are bit-identical to the batch without them (its slices and per-slice
    partials do not change)."""
    mats, bs, B = small_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    off = np.asarray(B.sys_row_off)
    x0, it0, st0, _, _ = mw.cg_solve_batched(arith, Ad, off, dev(B.b), tol=1e-12, maxit=20000)
    empty_at = [0, 0, 5, 11, len(off) - 1, len(off) - 1]   # before system k: a zero-row system
    off2 = np.insert(off, empty_at, off[empty_at])
    keep = np.ones(len(off2) - 1, dtype=bool)
    for j, k in enumerate(empty_at):
        keep[k + j] = False
    assert (np.diff(off2)[~keep] == 0).all() and (off2[1:][keep] == off[1:]).all()
    x1, it1, st1, rel1, _ = mw.cg_solve_batched(arith, Ad, off2, dev(B.b), tol=1e-12, maxit=20000)
    assert (it1[~keep] == 0).all() and (st1[~keep] == 0).all() and (rel1[~keep] == 0).all()
    assert np.array_equal(it1[keep], it0) and np.array_equal(st1[keep], st0)
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x0.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("arith", ["fp64", "dw", "qtw", "mxqtw"])
def test_batched_initial_guess(mw, small_batch, arith):
    """A nonzero x0 (random planes, per system r0 = b - A x0): per system
    the oracle's status, iterations within 2 % and true residual within 10x
    of the oracle started from the same x0."""
    mats, bs, _ = small_batch
    keep = [s for s in range(12) if np.any(bs[s])]   # with b = 0, x0 != 0 has no relative residual
    mats, bs = [mats[s] for s in keep], [bs[s] for s in keep]
    B = P.batch_from_systems(mats, bs)
    k = mw.WORDS[arith]
    x0 = rand_mw(np.random.default_rng(23), k, B.A.n, emin=-2, emax=2)
    xg, iters, status, _, _ = mw.cg_solve_batched(arith, mw.DeviceCSR.from_host(B.A), B.sys_row_off, dev(B.b),
                                                  x=dev(x0), tol=1e-12, maxit=20000)
    xg = xg.cpu().numpy()
    off = B.sys_row_off
    base = MIXED.get(arith, arith)
    for s, (A, b) in enumerate(zip(mats, bs)):
        xs = x0[:, off[s]:off[s + 1]]
        xo, io = O.cg_solve(base, A, b, x0=xs, tol=1e-12, maxit=20000, mixed=arith in MIXED)
        assert mw.STATUS[int(status[s])] == io["status"], (s, status[s], io)
        assert abs(int(iters[s]) - io["iters"]) <= max(1, int(0.02 * io["iters"])), (s, iters[s], io["iters"])
        nb = np.linalg.norm(b)
        tr_arith = "fp64" if arith in MIXED else arith
        trg = O.true_residual(tr_arith, A, b, xg[:, off[s]:off[s + 1]]) / nb
        tro = O.true_residual(tr_arith, A, b, xo) / nb
        assert trg <= 10 * max(tro, 1e-300), (s, trg, tro)


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_batched_bits_do_not_depend_on_chunk_length(mw, small_batch, arith):
    """Iterations per captured graph (1, 5, 16, 64) change only when the
    host polls and the running-slice list is rebuilt: x, iterations and
    status are bit-identical."""
    mats, bs, B = small_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    runs = [mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=20000, chunk=c)
            for c in (1, 5, 16, 64)]
    x0, it0, st0, _, _ = runs[0]
    for x, it, st, _, _ in runs[1:]:
        assert np.array_equal(it, it0) and np.array_equal(st, st0)
        assert np.array_equal(x.cpu().numpy().view(np.uint64), x0.cpu().numpy().view(np.uint64))


def test_batched_maxit(mw, small_batch):
    mats, bs, B = small_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    _, iters, status, _, info = mw.cg_solve_batched("dw", Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=5)
    for s in range(len(mats)):
        if s == 3:
            assert iters[s] == 0 and status[s] == 0
        elif s == len(mats) - 2:          # 1x1 system converges in one step
            assert iters[s] == 1 and status[s] == 0
        elif s == len(mats) - 1:
            assert status[s] == 2
        else:
            assert iters[s] == 5 and status[s] == 1


@pytest.fixture(scope="module")
def pcg_batch(small_batch):
    """The small batch plus systems whose diagonals vary: the scaled banded
    matrix (Jacobi undoes its D A D scaling), two shifted Laplacians, and a
    system with a zero diagonal entry (d_i = inf: breakdown at once)."""
    mats, bs, _ = small_batch
    mats, bs = list(mats), list(bs)
    A, b = P.case_banded_illcond(n=2048)[:2]
    mats.append(A)
    bs.append(b)
    for seed in (12, 13):
        L = P.poisson2d(20, 17).to_scipy().tolil()
        rng = np.random.default_rng(seed)
        for i in range(L.shape[0]):
            L[i, i] = L[i, i] + rng.uniform(0.0, 3.0)
        L = P.CSR.from_scipy(L.tocsr())
        mats.append(L)
        bs.append(L.matvec(rng.uniform(-1, 1, L.n)))
    mats.append(P.CSR.from_scipy(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 2.0]]))))
    bs.append(np.array([1.0, 1.0]))
    return mats, bs, P.batch_from_systems(mats, bs)


@pytest.mark.parametrize("arith", ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw", "mxdw", "mxqtw"])
def test_batched_jacobi_matches_oracle_per_system(mw, pcg_batch, arith):
    """Jacobi-preconditioned batch against the oracle's preconditioned CG run
    system by system: same status, iterations within 2 %, true residual
    within 10x; graph replay and direct launches give the same bits."""
    mats, bs, B = pcg_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    x, iters, status, rel, info = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-10, maxit=20000,
                                                      precond="jacobi")
    x2, iters2, _, _, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-10, maxit=20000,
                                              precond="jacobi", graph=False)
    assert np.array_equal(iters, iters2)
    assert np.array_equal(x.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))
    x = x.cpu().numpy()
    off = B.sys_row_off
    va = "fp64" if arith in MIXED else arith  # the arithmetic of the stored x
    for s, (A, b) in enumerate(zip(mats, bs)):
        if arith in MIXED:
            xo, io = O.cg_solve(MIXED[arith], A, b, tol=1e-10, maxit=20000, precond="jacobi", mixed=True)
        else:
            xo, io = O.cg_solve(arith, A, b, tol=1e-10, maxit=20000, precond="jacobi")
        st = {0: "ok", 1: "not_converged", 2: "breakdown"}[int(status[s])]
        assert st == io["status"], (s, st, io)
        assert abs(int(iters[s]) - io["iters"]) <= max(1, int(0.02 * io["iters"])), (s, iters[s], io["iters"])
        if io["status"] == "ok" and np.any(b):
            xs = x[:, off[s]:off[s + 1]]
            nb = np.linalg.norm(b)
            trg = O.true_residual(va, A, b, xs) / nb
            tro = O.true_residual(va, A, b, xo) / nb
            assert trg <= 10 * max(tro, 1e-300), (s, trg, tro)
    assert int(status[-1]) == 2 and int(iters[-1]) == 0        # zero diagonal entry
    # the scaled banded system: Jacobi converges where plain CG stalls
    nb_idx = len(bs) - 4
    assert int(status[nb_idx]) == 0 and int(iters[nb_idx]) < 100


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_batched_jacobi_diagonal_four_is_plain_cg(mw, arith):
    """2D Poisson systems (diagonal 4, M^-1 = I/4 exactly): the preconditioned
    batch reproduces the plain batch bit for bit."""
    mats = [P.poisson2d(nx, ny) for nx, ny in ((12, 9), (30, 31), (7, 40), (64, 64))]
    bs = [A.matvec(np.random.default_rng(s).uniform(-1, 1, A.n)) for s, A in enumerate(mats)]
    B = P.batch_from_systems(mats, bs)
    Ad = mw.DeviceCSR.from_host(B.A)
    x1, i1, s1, r1, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12)
    x2, i2, s2, r2, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12, precond="jacobi")
    assert np.array_equal(i1, i2) and np.array_equal(s1, s2) and np.array_equal(r1, r2)
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_batched_reuse_with_other_sparsity(mw, arith):
    """Two batched solves with the same system split, the same n, one shared
    workspace and one shared x, but a different number of stored entries:
    the slice copy moves inside the workspace, so the second solve must not
    replay the chunk captured for the first.  Each solve against the oracle
    per system (status, iterations within 2 %, true residual within 10x)."""
    import torch
    sizes = (400, 900, 256)
    first = [P.poisson2d(20), P.poisson2d(30), P.poisson2d(16)]
    second = [P.circulant_laplacian(n, offs, w) for n, offs, w in
              ((400, (1, 7, 20, 33), (0.5, 0.3, 0.9, 0.2)), (900, (1, 3, 30, 31, 100), (0.7, 0.2, 0.4, 0.6, 0.1)),
               (256, (1, 2, 16, 50, 77, 90), (0.3, 0.3, 0.5, 0.8, 0.2, 0.6)))]
    batches = []
    for mats in (first, second):
        assert tuple(m.n for m in mats) == sizes
        bs = [m.matvec(np.random.default_rng(40 + s).uniform(-1, 1, m.n)) for s, m in enumerate(mats)]
        batches.append((mats, bs, P.batch_from_systems(mats, bs)))
    assert batches[0][2].A.nnz != batches[1][2].A.nnz
    nbytes = max(mw.lib().mw_cg_batched_workspace_bytes(mw.ARITH[arith], 3, B.A.n, B.A.nnz) for _, _, B in batches)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    n = batches[0][2].A.n
    x = torch.zeros((mw.words(arith), n), dtype=torch.float64, device="cuda")
    for mats, bs, B in batches + batches[:1]:
        x.zero_()
        Ad = mw.DeviceCSR.from_host(B.A)
        xg, iters, status, _, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), x=x, tol=1e-12,
                                                      maxit=20000, workspace=ws)
        xg = xg.cpu().numpy()
        off = B.sys_row_off
        for s, (A, b) in enumerate(zip(mats, bs)):
            xo, io = O.cg_solve(arith, A, b, tol=1e-12, maxit=20000)
            assert int(status[s]) == 0 and io["status"] == "ok", (s, status[s], io)
            assert abs(int(iters[s]) - io["iters"]) <= max(1, int(0.02 * io["iters"])), (s, iters[s], io["iters"])
            nb = np.linalg.norm(b)
            trg = O.true_residual(arith, A, b, xg[:, off[s]:off[s + 1]]) / nb
            tro = O.true_residual(arith, A, b, xo) / nb
            assert trg <= 10 * tro, (s, trg, tro)


def _arrow(n, seed):
    """SPD arrow: tridiag(-1, 3, -1) plus a dense first row and column
    (weights U[0.1, 0.5]) and a first diagonal entry that dominates them."""
    rng = np.random.default_rng(seed)
    M = sp.diags([-np.ones(n - 1), 3.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    w = rng.uniform(0.1, 0.5, n - 1)
    M[0, 1:] = w
    M[1:, 0] = w.reshape(-1, 1)
    M[0, 0] = 2.0 * (w.sum() + 2.0)
    return P.CSR.from_scipy(M.tocsr())


@pytest.fixture(scope="module")
def long_row_batch():
    """Systems whose slices take vector rows: an arrow (one row of n entries
    in an otherwise tridiagonal matrix; SELL-64 would pad that slice to 64
    such rows) and a banded system of 81 entries per row, among Poisson and
    circulant systems that keep SELL-64."""
    mats = [P.poisson2d(20, 15), _arrow(2000, 1), P.banded_spd(1500, half_bw=40, seed=2, dseed=3, scale=False),
            P.circulant_laplacian(700, [1, 9, 50], [0.5, 0.8, 0.3]), _arrow(300, 4)]
    bs = [m.matvec(np.random.default_rng(60 + s).uniform(-1, 1, m.n)) for s, m in enumerate(mats)]
    return mats, bs, P.batch_from_systems(mats, bs)


def _per_system(arith, mats, bs, B, x, iters, status, tol):
    off = B.sys_row_off
    va = "fp64" if arith in MIXED else arith
    for s, (A, b) in enumerate(zip(mats, bs)):
        if arith in MIXED:
            xo, io = O.cg_solve(MIXED[arith], A, b, tol=tol, maxit=20000, mixed=True)
        else:
            xo, io = O.cg_solve(arith, A, b, tol=tol, maxit=20000)
        assert int(status[s]) == 0 and io["status"] == "ok", (s, status[s], io)
        assert abs(int(iters[s]) - io["iters"]) <= max(1, int(0.02 * io["iters"])), (s, iters[s], io["iters"])
        nb = np.linalg.norm(b)
        trg = O.true_residual(va, A, b, x[:, off[s]:off[s + 1]]) / nb
        tro = O.true_residual(va, A, b, xo) / nb
        assert trg <= 10 * max(tro, 1e-300), (s, trg, tro)


@pytest.mark.parametrize("arith", ["fp64", "dw", "qtw", "qqw", "mxqtw"])
def test_batched_vector_row_slices(mw, long_row_batch, arith):
    """Vector-row slices (long or very uneven rows) against the oracle per
    system, with the lanes per row of each slice's rule and with 4 and 64
    forced; graph replay and direct launches give the same bits."""
    mats, bs, B = long_row_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    for lanes in (None, 4, 64):
        shape = {"lanes": lanes} if lanes else None
        x, iters, status, _, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=20000,
                                                     shape=shape)
        x2, iters2, _, _, _ = mw.cg_solve_batched(arith, Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=20000,
                                                  shape=shape, graph=False)
        assert np.array_equal(iters, iters2)
        assert np.array_equal(x.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))
        _per_system(arith, mats, bs, B, x.cpu().numpy(), iters, status, 1e-12)


def test_batched_tuner_sweeps_lanes_of_vector_slices(mw, long_row_batch):
    mats, bs, B = long_row_batch
    Ad = mw.DeviceCSR.from_host(B.A)
    tuned_before, _ = mw.cg_shape("dw", B.A.n, B.A.nnz, nsys=B.nsys)
    assert not tuned_before
    best = mw.cg_batched_tune("dw", Ad, B.sys_row_off, dev(B.b), iters=8)
    assert best["lanes"] in (0, 2, 4, 8, 16, 32, 64) and best["spmv_grid"] > 0
    tuned, now = mw.cg_shape("dw", B.A.n, B.A.nnz, nsys=B.nsys)
    assert tuned and now["lanes"] == best["lanes"] and now["spmv_grid"] == best["spmv_grid"]
    x, iters, status, _, _ = mw.cg_solve_batched("dw", Ad, B.sys_row_off, dev(B.b), tol=1e-12, maxit=20000)
    _per_system("dw", mats, bs, B, x.cpu().numpy(), iters, status, 1e-12)
