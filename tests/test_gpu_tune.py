"""Launch shapes and the autotuners (mw_cg_tune, mw_cg_batched_tune) on the
GPU: a tuned or explicit shape changes only launch geometry, so the solves
keep the oracle-parity bar (single system) or stay bit-identical (batched,
whose reductions are per slice whatever the grid)."""
import numpy as np
import pytest

import oracle as O
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


def check_parity(arith, A, b, x_gpu, info, oinfo):
    assert info["status"] == oinfo["status"] == "ok"
    assert abs(info["iters"] - oinfo["iters"]) <= max(1, int(0.02 * oinfo["iters"]))
    xg = x_gpu.cpu().numpy()
    tr_g = O.true_residual(arith, A, b, xg)
    xo, _ = O.cg_solve(arith, A, b, tol=1e-12)
    tr_o = O.true_residual(arith, A, b, xo)
    assert tr_g <= 10 * max(tr_o, 1e-300), (tr_g, tr_o)


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_tuned_shape_is_recorded_and_used(mw, arith):
    # 80^3 rows: 2000 SpMV tiles and 2000 update blocks, so every candidate
    # grid (clamped at 2000) is a distinct launch
    A = P.poisson3d(80)
    rng = np.random.default_rng(3)
    b = A.matvec(rng.uniform(-1, 1, A.n))
    Ad = mw.DeviceCSR.from_host(A)
    bd = dev(b)
    tuned_before, builtin = mw.cg_shape(arith, A.n, A.nnz)
    assert not tuned_before
    best = mw.cg_tune(arith, Ad, bd, iters=16)
    assert best["spmv_grid"] in (1024, 1280, 1536, 1792, 2000)
    assert best["update_grid"] in (512, 1024, 2000)
    assert best["update_threads"] == 256 and best["us_per_iteration"] > 0
    tuned, now = mw.cg_shape(arith, A.n, A.nnz)
    assert tuned and now["spmv_grid"] == best["spmv_grid"] and now["update_grid"] == best["update_grid"]
    x1, i1 = mw.cg_solve(arith, Ad, bd, tol=1e-12)                    # the tuned shape
    x2, i2 = mw.cg_solve(arith, Ad, bd, tol=1e-12, shape=builtin)     # the built-in one, explicitly
    assert i1["status"] == i2["status"] == "ok"
    assert abs(i1["iters"] - i2["iters"]) <= max(1, int(0.02 * i2["iters"]))


@pytest.mark.parametrize("arith", ["fp64", "qtw"])
def test_tuner_sweeps_lanes_of_vector_rows(mw, arith):
    """A matrix the solver gives vector rows (3000 rows of ~37 entries:
    4 lanes in QTW, 8 in FP64 by the built-in rule): the tuner also tries
    half and twice the lanes; the winner is recorded and used, and the
    solve keeps the oracle-parity bar (5 % iterations in FP64: the rows are
    summed in another order than the oracle's)."""
    import scipy.sparse as sp
    n = 3000
    Bm = sp.random(n, n, density=6 / n, random_state=np.random.default_rng(9), format="csr")
    A = P.CSR.from_scipy((Bm.T @ Bm + 0.01 * sp.eye(n)).tocsr())
    b = A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n))
    Ad = mw.DeviceCSR.from_host(A)
    bd = dev(b)
    tuned, before = mw.cg_shape(arith, A.n, A.nnz)
    assert not tuned and before["lanes"] == (8 if arith == "fp64" else 4)
    best = mw.cg_tune(arith, Ad, bd, iters=16)
    L = before["lanes"]
    assert best["lanes"] in (L // 2, L, 2 * L) and best["us_per_iteration"] > 0
    tuned, now = mw.cg_shape(arith, A.n, A.nnz)
    assert tuned and now["lanes"] == best["lanes"]
    x, info = mw.cg_solve(arith, Ad, bd, tol=1e-12)
    xo, oinfo = O.cg_solve(arith, A, b, tol=1e-12)
    assert info["status"] == oinfo["status"] == "ok"
    slack = 0.05 if arith == "fp64" else 0.02
    assert abs(info["iters"] - oinfo["iters"]) <= max(1, int(slack * oinfo["iters"]))
    assert O.true_residual(arith, A, b, x.cpu().numpy()) <= 10 * O.true_residual(arith, A, b, xo)


@pytest.mark.parametrize("arith", ["dw", "qtw"])
def test_explicit_shape_keeps_parity(mw, arith):
    A, b, _ = P.case_poisson3d(nx=40)
    Ad = mw.DeviceCSR.from_host(A)
    bd = dev(b)
    _, oinfo = O.cg_solve(arith, A, b, tol=1e-12)
    shape = {"spmv_grid": 8, "update_grid": 8, "update_threads": 1024, "chunk": 6}
    x1, i1 = mw.cg_solve(arith, Ad, bd, tol=1e-12, shape=shape)
    x2, i2 = mw.cg_solve(arith, Ad, bd, tol=1e-12, shape=shape)
    check_parity(arith, A, b, x1, i1, oinfo)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))


def test_invalid_shape_rejected(mw):
    A, b, _ = P.case_poisson2d_64()
    with pytest.raises(mw.MWError):
        mw.cg_solve("dw", mw.DeviceCSR.from_host(A), dev(b), shape={"update_threads": 300})


def test_tuner_rejects_zero_rhs(mw):
    A = P.poisson2d(16)
    with pytest.raises(mw.MWError):
        mw.cg_tune("qtw", mw.DeviceCSR.from_host(A), dev(np.zeros(A.n)), iters=8)


def test_batched_tuner_and_grid_independence(mw):
    B = P.batch_systems(nsys=24, seed=12, nmin=200, nmax=4000)
    Ad = mw.DeviceCSR.from_host(B.A)
    bd = dev(B.b)
    ref = mw.cg_solve_batched("qtw", Ad, B.sys_row_off, bd, tol=1e-12, shape={"spmv_grid": 8, "chunk": 4})
    best = mw.cg_batched_tune("qtw", Ad, B.sys_row_off, bd, iters=8)
    assert best["spmv_grid"] in (256, 512, 1024, 1536, 2048) and best["us_per_iteration"] > 0
    tuned, now = mw.cg_shape("qtw", B.A.n, B.A.nnz, len(B.sys_row_off) - 1)
    assert tuned and now["spmv_grid"] == best["spmv_grid"]
    if best["lanes"]:  # lanes per row of vector-row slices set the row association: compare like with like
        ref = mw.cg_solve_batched("qtw", Ad, B.sys_row_off, bd, tol=1e-12,
                                  shape={"spmv_grid": 8, "chunk": 4, "lanes": best["lanes"]})
    got = mw.cg_solve_batched("qtw", Ad, B.sys_row_off, bd, tol=1e-12)   # tuned grid, default chunk
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    assert np.array_equal(got[0].cpu().numpy().view(np.uint64), ref[0].cpu().numpy().view(np.uint64))
    assert got[4]["status"] == "ok"


def test_tune_cache_file_carries_shapes_across_processes(tmp_path):
    """MW_TUNE_CACHE: what the tuner records in one process is the tuned
    shape of the next one (read at its first shape lookup); a line of
    another device is kept in the file but not applied, a malformed line is
    dropped."""
    import json
    import os
    import subprocess
    import sys
    repo = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    A = P.poisson3d(40)
    cache = tmp_path / "tune.jsonl"
    other = ('{"device": "gfx000/1", "arith": 1, "n": %d, "nnz": %d, "nsys": 0, "spmv_grid": 8, "update_grid": 8, '
             '"update_threads": 256, "chunk": 0, "lanes": 0, "us_per_iteration": 1.000000}' % (A.n, A.nnz))
    cache.write_text(other + "\nnot a cache line\n")
    env = dict(os.environ, MW_TUNE_CACHE=str(cache))
    pre = ("import json, numpy as np, torch; from paper_2510_13536_amd import mw, problems as P; "
           "A = P.poisson3d(40); ")
    tune = pre + ("Ad = mw.DeviceCSR.from_host(A); "
                  "b = torch.as_tensor(A.matvec(np.random.default_rng(3).uniform(-1, 1, A.n)), device='cuda'); "
                  "print(json.dumps([mw.cg_shape('dw', A.n, A.nnz)[0], mw.cg_tune('dw', Ad, b, iters=8)]))")
    look = pre + "print(json.dumps(mw.cg_shape('dw', A.n, A.nnz)))"
    for code in (tune, look):
        print("subprocess:", code[-60:], flush=True)
        r = subprocess.run([sys.executable, "-c", code], env=env, cwd=repo, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        out = json.loads(r.stdout.strip().splitlines()[-1])
        if code is tune:
            tuned_before, best = out
            assert not tuned_before                       # the other device's line is not applied
        else:
            tuned, now = out
    assert tuned and all(now[f] == best[f] for f in ("spmv_grid", "update_grid", "update_threads", "lanes"))
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[0] == other and '"arith": 1' in lines[1] and '"gfx000/1"' not in lines[1]
