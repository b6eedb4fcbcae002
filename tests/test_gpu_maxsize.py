"""The largest sizes the library takes, n = nnz = MW_MAX_N = 2^31 - 2^16,
built on the device: an FP64 CG solve of a diagonal system with that many
rows (its SELL-64 plan, SpMV, updates and reductions; about 190 GB of the
GPU's memory at the peak), a QTW dot and an FP64 gradient over that length.
Every 32-bit index a kernel forms there stays in range, so the results are
the exact ones."""
import pytest

pytestmark = pytest.mark.gpu

N = 2 ** 31 - 2 ** 16


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw as M
    M.lib()
    assert M.MAX_N == N
    return torch, M


def _need(torch, gb):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < gb * 1e9:
        pytest.skip("needs %d GB of free device memory, %.0f GB free" % (gb, free / 1e9))


def _diag(torch, mw, n, value):
    # column j of row j: col_idx shares row_ptr's first n entries
    row_ptr = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    return mw.DeviceCSR(n, row_ptr, row_ptr[:n], torch.full((n,), value, dtype=torch.float64, device="cuda"))


def test_fp64_cg_on_a_diagonal_system_of_max_n_rows(mods):
    torch, mw = mods
    _need(torch, 215)
    A = _diag(torch, mw, N, 2.0)
    b = torch.arange(N, dtype=torch.float64, device="cuda").remainder_(7).add_(1.0)
    x, info = mw.cg_solve("fp64", A, b, tol=1e-12, maxit=5)
    assert info["status"] == "ok" and info["iters"] == 1, info
    # b holds integers 1 .. 7: every partial sum of rho = b^T b and of
    # p^T q = 2 b^T b is an integer below 2^53, so alpha = 1/2, x = b / 2 and
    # r = 0 exactly, whatever the order of the sums
    assert torch.equal(x.reshape(-1), 0.5 * b)
    del A, b, x
    torch.cuda.empty_cache()


def test_qtw_dot_of_max_n(mods):
    torch, mw = mods
    _need(torch, 110)
    v = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    v[0] = 1.0
    d = mw.dot("qtw", v, v).cpu().tolist()
    assert d == [float(N), 0.0, 0.0], d
    del v
    torch.cuda.empty_cache()


def test_fp64_gradient_on_max_nnz(mods):
    torch, mw = mods
    _need(torch, 70)
    A = _diag(torch, mw, N, 2.0)
    lam = torch.ones((1, N), dtype=torch.float64, device="cuda")
    x = torch.full((1, N), 0.5, dtype=torch.float64, device="cuda")
    g = mw.csr_grad("fp64", A, lam, x)
    assert g.numel() == N and torch.all(g == -0.5).item()
    del A, lam, x, g
    torch.cuda.empty_cache()
