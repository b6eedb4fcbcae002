"""mw_dot_noalloc (the dot for callers that cannot allocate device memory)
against mw_dot, the entry point with a caller-provided workspace: same
kernels and summation order, so the two results must be bit-identical in
every arithmetic; each is also held to the dot's bound against the exact
value.  Two calls in a row, the second on a smaller input, so the second
runs over partial sums the first left in the shared scratch array."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from conftest import rand_mw

pytestmark = pytest.mark.gpu

ARITHS = ["fp64", "dw", "qdw", "tw", "qtw", "qtwe"]
DOT_BOUND = {1: 2.0 ** -45, 2: 2.0 ** -100, 3: 2.0 ** -145}
MAX_N = 33554432  # MW_DOT_NOALLOC_MAX_N


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw as M
    L = M.lib()
    L.mw_dot_noalloc.argtypes = [C.c_int, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    return M


def dot_noalloc_abi(M, arith, x, y):
    """Calls mw_dot_noalloc through the C ABI; returns (status, result)."""
    import torch
    k = M.WORDS[arith]
    n = x.shape[1]
    out = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    rc = M.lib().mw_dot_noalloc(M.ARITH[arith], n, x.data_ptr(), y.data_ptr(), out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc, out.cpu().numpy()


def dot_ws_abi(M, arith, x, y):
    """mw_dot with its own workspace through the C ABI."""
    import torch
    k = M.WORDS[arith]
    n = x.shape[1]
    L = M.lib()
    ws = torch.empty(L.mw_dot_workspace_bytes(M.ARITH[arith], n), dtype=torch.uint8, device="cuda")
    out = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    rc = L.mw_dot(M.ARITH[arith], n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                  C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0
    return out.cpu().numpy()


@pytest.mark.parametrize("arith", ARITHS)
def test_two_calls_second_smaller(mw, arith):
    import torch
    k = mw.WORDS[arith]
    for n, seed in ((1_000_003, 1), (4_099, 2)):
        rng = np.random.default_rng(seed)
        xh = rand_mw(rng, k, n, emin=-6, emax=6)
        yh = rand_mw(rng, k, n, emin=-6, emax=6)
        x = torch.as_tensor(xh, device="cuda")
        y = torch.as_tensor(yh, device="cuda")
        rc, d = dot_noalloc_abi(mw, arith, x, y)
        assert rc == 0, mw.lib().mw_last_error()
        ref = dot_ws_abi(mw, arith, x, y)
        assert np.array_equal(d, ref), (n, d, ref)
        err, sc = O.dot_error(arith, xh, yh, d)
        assert err <= DOT_BOUND[k] * sc, (n, err / sc)


def test_at_the_maximum_size_then_small(mw):
    """n = MW_DOT_NOALLOC_MAX_N (every scratch slot in use), then n = 300."""
    import torch
    for n in (MAX_N, 300):
        g = torch.Generator(device="cuda").manual_seed(n)
        x = torch.rand((3, n), dtype=torch.float64, device="cuda", generator=g) - 0.5
        y = torch.rand((3, n), dtype=torch.float64, device="cuda", generator=g) - 0.5
        x[1:] *= 2.0 ** -60
        y[1:] *= 2.0 ** -60
        rc, d = dot_noalloc_abi(mw, "qtw", x, y)
        assert rc == 0, mw.lib().mw_last_error()
        assert np.array_equal(d, dot_ws_abi(mw, "qtw", x, y))
        del x, y


def test_empty_and_too_large(mw):
    import torch
    z = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    rc, d = dot_noalloc_abi(mw, "qtw", z, z)
    assert rc == 0 and np.all(d == 0.0)
    out = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    x = torch.zeros((3, 8), dtype=torch.float64, device="cuda")  # never read: rejected on the host
    rc = mw.lib().mw_dot_noalloc(mw.ARITH["qtw"], MAX_N + 1, x.data_ptr(), x.data_ptr(), out.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == -1
    assert b"MW_DOT_NOALLOC_MAX_N" in mw.lib().mw_last_error()
    assert np.all(out.cpu().numpy() == 7.0)
