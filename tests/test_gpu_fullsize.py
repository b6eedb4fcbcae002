"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (planned SELL-64 SpMV, graph-replayed CG chunks):

* 3D Poisson 128^3 and the banded ill-conditioned matrix (n = 2^20,
  27 per row): the whole SpMV bit-identical to the oracle, all arithmetics;
* the first 5 CG iterations match the oracle's iterate to near the
  format's precision (only the dot association differs);
* complete 128^3 solves in every arithmetic against the oracle's solve in
  the same arithmetic (stored results): iterations within 2 %, true
  residual within 10x;
* the largest vector-row workload (the banded stand-in of nd24k, 72,000
  rows of ~400 entries, with the plan the solver picks): sampled rows
  within the bound of the reassociated row sum, all arithmetics;
* the 512-system batch: small, median and the largest systems against
  oracle solves (live or stored);
* the adjoint problem at 100^3: gradients against central differences at
  64 + 64 coordinates, and against the oracle's gradient there.
"""
import numpy as np
import pytest

import oracle as O
from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu

ARITHS = ["fp64", "dw", "qdw", "tw", "qtw"]


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw
    mw.lib()
    return torch, mw


@pytest.fixture(scope="module")
def c2():
    return P.case_poisson3d(128)


@pytest.fixture(scope="module")
def c3():
    return P.case_banded_illcond()


def _rand_words(k, n, seed):
    rng = np.random.default_rng(seed)
    x = [rng.uniform(-1, 1, n)]
    for _ in range(1, k):
        x.append(x[-1] * rng.uniform(-1, 1, n) * 2.0 ** -54)
    return np.ascontiguousarray(np.stack(x))


MIXED = {"mxdw": "dw", "mxqtw": "qtw"}


@pytest.mark.parametrize("case", ["c2", "c3"])
@pytest.mark.parametrize("arith", ARITHS + ["qtwe", "qw", "qqw", "mxdw", "mxqtw"])
def test_full_spmv_bit_exact(mods, request, case, arith):
    """Every row of the planned SpMV at full size bit for bit (the mixed
    types: the oracle's base-arithmetic row of the FP64 vector, rounded
    once to FP64)."""
    torch, mw = mods
    A = request.getfixturevalue(case)[0]
    plan = mw.Plan(mw.DeviceCSR.from_host(A))
    assert plan.format == "sell64"
    if arith in MIXED:
        base = MIXED[arith]
        x = _rand_words(1, A.n, 21)
        xp = np.zeros((O.WORDS[base], A.n))
        xp[0] = x[0]
        want = O.elementwise(base, "tofp64", O.spmv(base, A, xp)).reshape(1, -1)
    else:
        x = _rand_words(O.WORDS[arith], A.n, 21)
        want = O.spmv(arith, A, x)
    got = mw.spmv_planned(arith, plan, torch.as_tensor(x, device="cuda")).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.fixture(scope="module")
def nd24k():
    return P.table1_standin("nd24k")


@pytest.mark.parametrize("arith", ARITHS + ["qtwe", "qw", "qqw"])
def test_full_vector_row_spmv_sampled(mods, nd24k, arith):
    torch, mw = mods
    A = nd24k
    k = O.WORDS[arith]
    x = _rand_words(k, A.n, 22)
    plan = mw.Plan(mw.DeviceCSR.from_host(A), solver=arith)
    assert plan.format == "csrvec" and plan.lanes in (32, 64)
    got = mw.spmv_planned(arith, plan, torch.as_tensor(x, device="cuda")).cpu().numpy()
    rows = np.random.default_rng(5).choice(A.n, 2000, replace=False)
    rows = np.concatenate([rows, [0, A.n - 1]])
    err, sc = O.spmv_error(arith, A, x, got, rows=rows)
    lens = np.diff(A.row_ptr)[rows]
    bound = 8 * (np.ceil(lens / plan.lanes) + np.log2(plan.lanes) + 2) * 2.0 ** (-53 * k) * sc
    assert np.all(err <= bound), np.max(err / bound)


def _word_diff(arith, a, b):
    """max_i |a_i - b_i| (exact word sums rounded) and max |b_i|."""
    d = O.elementwise(arith, "add", a, -b)
    return np.abs(O.elementwise(arith, "tofp64", d)).max(), np.abs(O.elementwise(arith, "tofp64", b)).max()


@pytest.mark.parametrize("case", ["c2", "c3"])
@pytest.mark.parametrize("arith", ["fp64", "dw", "qdw", "tw", "qtw", "qtwe", "qw", "qqw", "mxdw", "mxqtw"])
def test_first_iterations_match_oracle(mods, request, case, arith):
    torch, mw = mods
    A, b, _ = request.getfixturevalue(case)
    xg, ig = mw.cg_solve(arith, mw.DeviceCSR.from_host(A), torch.as_tensor(b, device="cuda"), tol=1e-30, maxit=5)
    if arith in MIXED:
        xo, io = O.cg_solve(MIXED[arith], A, b, tol=1e-30, maxit=5, mixed=True)
    else:
        xo, io = O.cg_solve(arith, A, b, tol=1e-30, maxit=5)
    assert ig["status"] == io["status"] == "not_converged" and ig["iters"] == io["iters"] == 5
    diff, scale = _word_diff("fp64" if arith in MIXED else arith, xg.cpu().numpy(), xo)
    # The iterates differ only through the association of the dots (tree on
    # the GPU, sequential in the oracle): an error of about n u^k
    # sum|p_i q_i| / |p^T q| in alpha and beta.  On the D A D-scaled banded
    # matrix the terms of p^T q span ~12 decades and cancel heavily, so its
    # bounds are wider; both stay far below the next-lower format's unit
    # round-off (multi-word differences are ~1e-20 below FP64's).
    # The quasi types' unnormalised intermediates leave them a little
    # further (measured on C3: QDW 1.5e-24, QQW 6.9e-49, against DW's and
    # QW's 1e-25 and 4.5e-63); the mixed types' x is FP64 (FP64's bounds;
    # measured: identical iterates).
    bound = {"c2": {"fp64": 1e-12, "mxdw": 1e-12, "mxqtw": 1e-12, "dw": 1e-26, "qdw": 1e-26, "tw": 1e-36,
                    "qtw": 1e-36, "qtwe": 1e-36, "qw": 1e-58, "qqw": 1e-50},
             "c3": {"fp64": 1e-10, "mxdw": 1e-10, "mxqtw": 1e-10, "dw": 1e-24, "qdw": 1e-22, "tw": 1e-34,
                    "qtw": 1e-34, "qtwe": 1e-34, "qw": 1e-56, "qqw": 1e-45}}[case][arith]
    assert diff <= bound * scale, (diff / scale)


def _golden(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)))


@pytest.mark.parametrize("arith", ARITHS + ["qw", "qqw", "qtwe", "mxdw", "mxqtw"])
def test_c2_full_solve(mods, c2, arith):
    """The whole 128^3 solve against the oracle's solve in the same
    arithmetic (stored by tests/golden/make_fullsize_oracle.py, which runs
    only the oracle; the mixed types against its mixed solve): same status,
    iterations within 2 %, true residual (formed exactly) within 10x of the
    oracle's."""
    torch, mw = mods
    A, b, _ = c2
    ref = _golden("c2_oracle_solves.json")
    assert (ref["n"], ref["nnz"]) == (A.n, A.nnz)
    io = ref["solves"][arith]
    xg, ig = mw.cg_solve(arith, mw.DeviceCSR.from_host(A), torch.as_tensor(b, device="cuda"), tol=1e-12)
    assert ig["status"] == io["status"] == "ok" and ig["rel_res"] < 1e-12
    assert abs(ig["iters"] - io["iters"]) <= max(1, int(0.02 * io["iters"])), (ig, io)
    nb = np.linalg.norm(b)
    va = "fp64" if arith in ("mxdw", "mxqtw") else arith  # the mixed types' x is FP64
    tr = O.true_residual(va, A, b, xg.cpu().numpy()) / nb
    assert tr <= 10 * io["true_rel_res"], (tr, io["true_rel_res"])


def test_true_residual_helper_matches_oracle(mods, c2):
    """The benchmark's true-residual helper (product and difference in QTW,
    dots in TW, on the GPU) against the oracle's exactly formed residual,
    for a QTW solution at 1e-24 and for its leading words alone (an FP64
    vector)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    torch, mw = mods
    A, b, _ = c2
    Ad = mw.DeviceCSR.from_host(A)
    bd = torch.as_tensor(b, device="cuda")
    xg, ig = mw.cg_solve("qtw", Ad, bd, tol=1e-24)
    assert ig["status"] == "ok"
    nb = np.linalg.norm(b)
    for x in (xg, xg[:1].contiguous()):
        got = bench.true_rel_residual(mw, torch, Ad, bd, x)
        want = O.true_residual("qtw" if x.shape[0] == 3 else "fp64", A, b, x.cpu().numpy()) / nb
        assert abs(got - want) <= 1e-6 * want, (got, want)


@pytest.mark.parametrize("arith", ["qtw", "dw"])
def test_c4_batch_sampled_systems(mods, arith):
    """The 512-system batch in one batched solve: about a dozen small
    systems against live oracle solves, and the four largest and four of
    median size against the oracle's solves stored by
    tests/golden/make_fullsize_oracle.py; each: same status, iterations
    within 2 %, true residual within 10x of the oracle's."""
    torch, mw = mods
    B = P.batch_systems()
    Ad = mw.DeviceCSR.from_host(B.A)
    x, iters, status, rel, info = mw.cg_solve_batched(arith, Ad, B.sys_row_off,
                                                      torch.as_tensor(B.b, device="cuda"), tol=1e-12)
    assert (status == 0).all()
    x = x.cpu().numpy()
    sizes = np.diff(B.sys_row_off)

    def check(s, io_iters, io_true):
        A, b = B.system(s)
        assert abs(int(iters[s]) - io_iters) <= max(1, int(0.02 * io_iters)), (s, iters[s], io_iters)
        r0, r1 = B.sys_row_off[s], B.sys_row_off[s + 1]
        tr = O.true_residual(arith, A, b, x[:, r0:r1]) / np.linalg.norm(b)
        assert tr <= 10 * max(io_true, 1e-300), (s, tr, io_true)

    small = [s for s in range(B.nsys) if sizes[s] <= 2500]
    for s in small[:: max(1, len(small) // 12)]:
        A, b = B.system(s)
        xo, io = O.cg_solve(arith, A, b, tol=1e-12)
        assert io["status"] == "ok"
        check(s, io["iters"], O.true_residual(arith, A, b, xo) / np.linalg.norm(b))
    ref = _golden("c4_oracle_solves.json")["systems"]
    assert len(ref) == 8
    for s, rec in ref.items():
        s = int(s)
        assert sizes[s] == rec["n"]
        assert rec[arith]["status"] == "ok"
        check(s, rec[arith]["iters"], rec[arith]["true_rel_res"])


def test_c5_adjoint_finite_differences(mods):
    """Adjoint gradients on 100^3 + diag(theta) against central differences
    at 64 random theta and 64 random b coordinates (seed 5555), every
    difference solve in QTW to 1e-24 (plan rebuilt inside each solve, one
    workspace); accept |g - g_fd| <= 1e-6 |g_fd| + 1e-9 ||g||_inf.  At the
    same coordinates the gradient equals the oracle's (its QTW solves to
    1e-26, stored) to 1e-10 relative."""
    torch, mw = mods
    from paper_2510_13536_amd import adjoint
    Q = P.adjoint_problem(nx=100)
    Ad = mw.DeviceCSR.from_host(Q.lap)
    theta = torch.as_tensor(Q.theta, device="cuda").requires_grad_(True)
    b = torch.as_tensor(Q.b, device="cuda").requires_grad_(True)
    xt = torch.as_tensor(Q.x_target, device="cuda")
    pos = torch.as_tensor(Q.diag_pos, device="cuda")
    val = torch.as_tensor(Q.lap.val, device="cuda").index_add(0, pos, theta)
    x = adjoint.cg_solve(Ad, val, b, arith="qtw", tol=1e-26)
    (0.5 * ((x - xt) ** 2).sum()).backward()
    g = theta.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()

    # one matrix and one right-hand side buffer, perturbed in place, so the
    # solver's captured chunk and workspace are reused across the solves
    val0 = val.detach().clone()
    vbuf = val0.clone()
    A = mw.DeviceCSR(Ad.n, Ad.row_ptr, Ad.col_idx, vbuf)
    b0 = torch.as_tensor(Q.b, device="cuda")
    bbuf = b0.clone()
    ws = mw.cg_workspace("qtw", A)
    xs = torch.zeros((3, A.n), dtype=torch.float64, device="cuda")
    t = torch.zeros_like(xs)
    t[0] = -xt

    def loss():
        xs.zero_()
        _, info = mw.cg_solve("qtw", A, bbuf, x=xs, tol=1e-24, workspace=ws)
        assert info["status"] == "ok"
        d = mw.elementwise("qtw", "add", xs, t)
        return mw.dot("qtw", d, d) * 0.5

    def diff(a, c):
        return float(mw.elementwise("qtw", "tofp64", mw.elementwise("qtw", "add", a.reshape(3, 1), -c.reshape(3, 1)))[0, 0])

    rng = np.random.default_rng(5555)
    ith = rng.choice(Q.lap.n, 64, replace=False)
    ib = rng.choice(Q.lap.n, 64, replace=False)
    gmax, gbmax = np.abs(g).max(), np.abs(gb).max()

    # the oracle's gradient at the same coordinates (its forward and adjoint
    # QTW solves to 1e-26, stored by tests/golden/make_fullsize_oracle.py)
    ref = _golden("c5_oracle_gradient.json")
    assert ref["forward"]["status"] == ref["adjoint"]["status"] == "ok"
    assert ref["theta_index"] == [int(i) for i in ith] and ref["b_index"] == [int(i) for i in ib]
    np.testing.assert_allclose(g[ith], ref["theta_grad"], rtol=1e-10, atol=1e-12 * ref["theta_grad_absmax"])
    np.testing.assert_allclose(gb[ib], ref["b_grad"], rtol=1e-10, atol=1e-12 * ref["b_grad_absmax"])
    assert abs(gmax - ref["theta_grad_absmax"]) <= 1e-10 * gmax and abs(gbmax - ref["b_grad_absmax"]) <= 1e-10 * gbmax
    for i in ith:
        h = 1e-4 * max(abs(Q.theta[i]), 1e-2)
        k = int(Q.diag_pos[i])
        vbuf.copy_(val0)
        vbuf[k] += h
        vp = float(vbuf[k])
        lp = loss()
        vbuf.copy_(val0)
        vbuf[k] -= h
        vm = float(vbuf[k])
        lm = loss()
        fd = diff(lp, lm) / (vp - vm)
        assert abs(g[i] - fd) <= 1e-6 * abs(fd) + 1e-9 * gmax, ("theta", i, g[i], fd)
    vbuf.copy_(val0)
    for i in ib:
        bbuf.copy_(b0)
        bbuf[i] += 1e-4
        bp = float(bbuf[i])
        lp = loss()
        bbuf.copy_(b0)
        bbuf[i] -= 1e-4
        bm = float(bbuf[i])
        lm = loss()
        fd = diff(lp, lm) / (bp - bm)
        assert abs(gb[i] - fd) <= 1e-6 * abs(fd) + 1e-9 * gbmax, ("b", i, gb[i], fd)
