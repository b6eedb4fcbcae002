"""GPU parity of the mixed-precision arithmetics MXDW / MXQTW (FP64
vectors, SpMV rows and dots accumulated in DW / QTW; Sec. VI names mixed
precision as future work) against the oracle's mixed reading:

* SpMV: every row bit-identical to the oracle's row accumulated in the base
  arithmetic from the promoted FP64 vector and rounded once to FP64;
* DOT: within the base format's bound of the exact dot of the FP64 vectors;
* AXPY: y = fma(fp64(alpha), x, y) bit for bit;
* CG: same status, iterations within 2 %, true residual within 10x of the
  oracle's mixed solve; the error against an exact solution stays FP64's;
* Jacobi PCG (z_i = fl(d_i r_i)) against the oracle's mixed PCG;
* the entry points that do not take the mixed types reject them (the
  element-wise ops, the gradient kernel).
"""
import numpy as np
import pytest

import oracle as O
from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu

MIXED = {"mxdw": "dw", "mxqtw": "qtw"}
DOT_BOUND = {"dw": 2.0 ** -100, "qtw": 2.0 ** -145}


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


def promote(x, k):
    out = np.zeros((k, x.size))
    out[0] = x
    return out


MATS = {
    "poisson2d_64": lambda: P.poisson2d(64),
    "banded27": lambda: P.banded_spd(5000, half_bw=13, seed=1, dseed=2),
    "circulant": lambda: P.circulant_laplacian(3001, [1, 17, 400, 1200], [0.5, 0.3, 1.0, 0.2]),
}


@pytest.mark.parametrize("arith", sorted(MIXED))
@pytest.mark.parametrize("mat", sorted(MATS))
@pytest.mark.parametrize("planned", [False, True])
def test_spmv_rows_rounded_once(mw, arith, mat, planned):
    base = MIXED[arith]
    k = O.WORDS[base]
    A = MATS[mat]()
    x = np.random.default_rng(31).uniform(-1, 1, A.n) * 2.0 ** np.random.default_rng(32).integers(-6, 6, A.n)
    want = O.elementwise(base, "tofp64", O.spmv(base, A, promote(x, k)))
    Ad = mw.DeviceCSR.from_host(A)
    if planned:
        got = mw.spmv_planned(arith, mw.Plan(Ad), dev(x.reshape(1, -1))).cpu().numpy()[0]
    else:
        got = mw.spmv(arith, Ad, dev(x.reshape(1, -1))).cpu().numpy()[0]
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("arith", sorted(MIXED))
@pytest.mark.parametrize("n", [1, 2049, 100003])
def test_dot_within_bound(mw, arith, n):
    base = MIXED[arith]
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    d = mw.dot(arith, dev(x.reshape(1, -1)), dev(y.reshape(1, -1))).cpu().numpy()
    assert d.size == O.WORDS[base]
    k = O.WORDS[base]
    err, sc = O.dot_error(base, promote(x, k), promote(y, k), d)
    assert err <= DOT_BOUND[base] * sc


@pytest.mark.parametrize("arith", sorted(MIXED))
def test_axpy_rounds_alpha_then_fma(mw, arith):
    base = MIXED[arith]
    rng = np.random.default_rng(7)
    n = 5001
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    al = np.array([0.3, 2.0 ** -55, 2.0 ** -110][:O.WORDS[base]])
    a64 = O.elementwise(base, "tofp64", al.reshape(-1, 1))[0]
    want = O.axpy("fp64", [a64], x.reshape(1, -1), y.reshape(1, -1))[0]
    yd = dev(y.reshape(1, -1))
    mw.axpy(arith, dev(al), dev(x.reshape(1, -1)), yd)
    assert np.array_equal(yd.cpu().numpy()[0].view(np.uint64), want.view(np.uint64))


def _cg_parity(mw, arith, A, b, tol, maxit=None, precond=None):
    base = MIXED[arith]
    xo, io = O.cg_solve(base, A, b, tol=tol, maxit=maxit, mixed=True, precond=precond)
    xg, ig = mw.cg_solve(arith, mw.DeviceCSR.from_host(A), dev(b), tol=tol, maxit=maxit, precond=precond)
    xg = xg.cpu().numpy()
    assert xg.shape == (1, A.n)
    assert ig["status"] == io["status"], (ig, io)
    assert abs(ig["iters"] - io["iters"]) <= max(1, int(0.02 * io["iters"])), (ig["iters"], io["iters"])
    nb = np.linalg.norm(b)
    tro = O.true_residual("fp64", A, b, xo) / nb
    trg = O.true_residual("fp64", A, b, xg) / nb
    assert trg <= 10 * max(tro, 1e-300), (trg, tro)
    return xg, ig


@pytest.mark.parametrize("arith", sorted(MIXED))
def test_cg_poisson2d_64(mw, arith):
    A, b, _ = P.case_poisson2d_64()
    _cg_parity(mw, arith, A, b, 1e-12)


@pytest.mark.parametrize("arith", sorted(MIXED))
def test_cg_banded_scaled_and_3d(mw, arith):
    A = P.banded_spd(6000, half_bw=13, seed=5, dseed=6)
    b = A.matvec(P.uniform(A.n, 7))
    _cg_parity(mw, arith, A, b, 1e-10, maxit=3000)
    A = P.poisson3d(20, 17, 13)
    _cg_parity(mw, arith, A, A.matvec(P.uniform(A.n, 8)), 1e-12)


@pytest.mark.parametrize("arith", sorted(MIXED))
def test_cg_accuracy_stays_fp64s(mw, arith):
    """The recursive residual reaches 1e-30, the error against an integer
    solution stays at FP64's level (x is FP64), as in the oracle."""
    A = P.poisson2d(40, 30)
    xs = P.integer_vector(A.n, seed=3)
    b = A.matvec(xs)
    xg, ig = _cg_parity(mw, arith, A, b, 1e-30, maxit=600)
    assert ig["status"] == "ok"
    err = np.abs(xg[0] - xs).max() / np.abs(xs).max()
    assert 1e-17 < err < 1e-13


@pytest.mark.parametrize("arith", sorted(MIXED))
def test_cg_jacobi(mw, arith):
    """Jacobi PCG with FP64 vectors (z_i = fl(d_i r_i)) against the oracle's
    mixed PCG: the scaled banded case it rescues, a shifted Laplacian with a
    varying diagonal; diagonal 4 reproduces the plain mixed solve bit for bit."""
    A, b, _ = P.case_banded_illcond(n=4096)
    xg, ig = _cg_parity(mw, arith, A, b, 1e-10, maxit=2000, precond="jacobi")
    assert ig["status"] == "ok" and ig["iters"] <= 60
    S = P.poisson2d(30, 27).to_scipy().tolil()
    rng = np.random.default_rng(12)
    for i in range(S.shape[0]):
        S[i, i] = S[i, i] + rng.uniform(0.0, 3.0)
    S = P.CSR.from_scipy(S.tocsr())
    _cg_parity(mw, arith, S, S.matvec(rng.uniform(-1, 1, S.n)), 1e-12, precond="jacobi")
    A, b, _ = P.case_poisson2d_64()
    Ad = mw.DeviceCSR.from_host(A)
    x1, i1 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12)
    x2, i2 = mw.cg_solve(arith, Ad, dev(b), tol=1e-12, precond="jacobi")
    assert i1["iters"] == i2["iters"] and i1["rel_res"] == i2["rel_res"]
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))


def test_other_entry_points_reject_mixed(mw):
    import torch
    A = P.poisson2d(8)
    Ad = mw.DeviceCSR.from_host(A)
    x = torch.zeros((1, A.n), dtype=torch.float64, device="cuda")
    with pytest.raises(mw.MWError):
        mw.elementwise("mxdw", "add", x, x)
    with pytest.raises(mw.MWError):
        mw.csr_grad("mxqtw", Ad, x, x)
    with pytest.raises(mw.MWError):
        mw.cg_solve("mxdw", Ad, dev(np.ones(A.n)), normalize_p=True, precond="jacobi")
    assert mw.lib().mw_words(8) == 1 and mw.lib().mw_scalar_words(9) == 3
