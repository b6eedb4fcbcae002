"""mw_csr_check (the device check of a CSR matrix's structure), the
MW_CHECK_CSR guard that runs it at every entry point, and non-finite
right-hand sides against the oracle.  The malformed matrices here are only
ever passed to the check itself, or to entry points under the guard, which
rejects them before any other kernel reads them."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle as O
from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw as M
    M.lib()
    return M


def _device_csr(mw, n, rp, ci, va):
    import torch
    return mw.DeviceCSR(n, torch.as_tensor(np.asarray(rp, dtype=np.int32), device="cuda"),
                        torch.as_tensor(np.asarray(ci, dtype=np.int32), device="cuda"),
                        torch.as_tensor(np.asarray(va, dtype=np.float64), device="cuda"))


def _broken(A, how):
    rp, ci = A.row_ptr.copy(), A.col_idx.copy()
    if how == "row_ptr_start":
        rp[0] = 1
    elif how == "row_ptr_end":
        rp[-1] = A.nnz - 1
    elif how == "row_ptr_decreasing":
        rp[A.n // 2] = rp[A.n // 2 + 1] + 1
    elif how == "column_n":
        ci[A.nnz // 3] = A.n
    elif how == "column_negative":
        ci[-1] = -1
    return rp, ci


BROKEN = {"row_ptr_start": r"row_ptr\[0\]", "row_ptr_end": r"row_ptr\[0\]", "row_ptr_decreasing": "decreases",
          "column_n": "column index", "column_negative": "column index"}


@pytest.mark.parametrize("how", list(BROKEN))
def test_csr_check_names_the_broken_property(mw, how):
    A = P.poisson3d(9, 8, 7)
    mw.csr_check(mw.DeviceCSR.from_host(A))            # the intact matrix passes
    rp, ci = _broken(A, how)
    with pytest.raises(mw.MWError, match=BROKEN[how]):
        mw.csr_check(_device_csr(mw, A.n, rp, ci, A.val))


def test_csr_check_on_wide_and_single_row_matrices(mw):
    for A in (P.table1_standin("pdb1HYS"), P.CSR.from_scipy(np.array([[2.0]]))):
        mw.csr_check(mw.DeviceCSR.from_host(A))


def test_guard_rejects_malformed_matrices_at_every_entry_point():
    """In a process with MW_CHECK_CSR=1: a column index n is refused by the
    solvers, the SpMVs, the plan builders, the gradient and the tuner before
    any of their kernels runs; an intact matrix still solves to the oracle's
    iteration count."""
    code = r'''
import json, numpy as np, torch
from paper_2510_13536_amd import mw, problems as P
A = P.poisson2d(20)
b = A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n))
bd = torch.as_tensor(b, device="cuda")
ci = A.col_idx.copy(); ci[A.nnz // 2] = A.n
bad = mw.DeviceCSR(A.n, torch.as_tensor(A.row_ptr, device="cuda"), torch.as_tensor(ci, device="cuda"),
                   torch.as_tensor(A.val, device="cuda"))
good = mw.DeviceCSR.from_host(A)
x = torch.zeros((3, A.n), dtype=torch.float64, device="cuda")
calls = {
    "cg_solve": lambda: mw.cg_solve("qtw", bad, bd),
    "cg_solve_batched": lambda: mw.cg_solve_batched("qtw", bad, [0, A.n], bd),
    "spmv": lambda: mw.spmv("qtw", bad, x),
    "plan": lambda: mw.Plan(bad),
    "cg_plan": lambda: mw.Plan(bad, solver="qtw"),
    "csr_grad": lambda: mw.csr_grad("qtw", bad, x, x),
    "cg_tune": lambda: mw.cg_tune("qtw", bad, bd, iters=8),
}
out = {}
for name, f in calls.items():
    try:
        f()
        out[name] = "accepted"
    except mw.MWError as e:
        out[name] = "column index" in str(e)
_, info = mw.cg_solve("qtw", good, bd, tol=1e-12)
out["good_iters"] = info["iters"]
print(json.dumps(out))
'''
    env = dict(os.environ, MW_CHECK_CSR="1")
    print("subprocess: MW_CHECK_CSR=1 entry points", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    A = P.poisson2d(20)
    b = A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n))
    _, io = O.cg_solve("qtw", A, b, tol=1e-12)
    assert out.pop("good_iters") == io["iters"]
    assert all(v is True for v in out.values()), out


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_non_finite_rhs_breaks_down_like_the_oracle(mw, bad, precond):
    A = P.poisson2d(12)
    b = np.ones(A.n)
    b[5] = bad
    Ad = mw.DeviceCSR.from_host(A)
    import torch
    for arith in ("fp64", "dw", "qtw"):
        _, io = O.cg_solve(arith, A, b, tol=1e-12, precond=precond)
        _, ig = mw.cg_solve(arith, Ad, torch.as_tensor(b, device="cuda"), tol=1e-12, precond=precond)
        assert ig["status"] == io["status"] == "breakdown" and ig["iters"] == io["iters"] == 0, (arith, ig, io)
        _, it, st, _, _ = mw.cg_solve_batched(arith, Ad, [0, A.n], torch.as_tensor(b, device="cuda"), tol=1e-12,
                                              precond=precond)
        assert int(st[0]) == 2 and int(it[0]) == 0, (arith, st, it)
