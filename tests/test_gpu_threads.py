"""Calls from several host threads at once.  The library keeps its streams,
captured graphs, pinned host buffers and error text per thread (streams
also per device), and the binding releases the interpreter lock during
each call, so solves running at the same time on two threads, each on a
stream of its own, give the same bits as the same solves run one after
another on one thread."""
import threading

import numpy as np
import pytest

from paper_2510_13536_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2510_13536_amd import mw as M
    M.lib()
    return torch, M


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_single_and_batched_solves_on_two_threads_match_one_thread(mods):
    torch, mw = mods
    single = []
    for arith, A, seed in [("qtw", P.poisson3d(40), 1), ("dw", P.poisson2d(96), 2),
                           ("fp64", P.banded_spd(20000, scale=False), 3), ("qtw", P.poisson2d(64), 4),
                           ("mxqtw", P.poisson3d(24), 5), ("qw", P.poisson2d(40), 6)]:
        b = A.matvec(np.random.default_rng(seed).uniform(-1.0, 1.0, A.n))
        single.append((arith, mw.DeviceCSR.from_host(A), _dev(torch, b)))
    B = P.batch_systems(nsys=24, seed=7, nmin=256, nmax=4096)
    batch = ("qtw", mw.DeviceCSR.from_host(B.A), B.sys_row_off, _dev(torch, B.b))

    def run(job):
        if job == "batch":
            arith, Ad, off, bd = batch
            x, iters, status, _, _ = mw.cg_solve_batched(arith, Ad, off, bd, tol=1e-12)
            return x.cpu().numpy(), iters.tolist(), status.tolist()
        arith, Ad, bd = single[job]
        x, info = mw.cg_solve(arith, Ad, bd, tol=1e-14)
        return x.cpu().numpy(), info["iters"], info["status"]

    jobs = list(range(len(single))) + ["batch"]
    expected = {j: run(j) for j in jobs}
    torch.cuda.synchronize()
    assert all(expected[j][2] == "ok" for j in range(len(single)))

    # thread 0 takes the even single solves and the batch, thread 1 the odd
    # ones; each repeats its list three times
    split = [[j for j in jobs if j == "batch" or j % 2 == 0], [j for j in jobs if j != "batch" and j % 2 == 1]]
    got = [[], []]
    errors = []
    start = threading.Barrier(2)

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                start.wait(timeout=60)
                for _ in range(3):
                    for j in split[t]:
                        got[t].append((j, run(j)))
        except BaseException as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(t,)) for t in (0, 1)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=300)
    assert not any(th.is_alive() for th in threads), "a solver thread did not finish"
    assert not errors, errors
    for t in (0, 1):
        assert len(got[t]) == 3 * len(split[t])
        for j, (x, iters, status) in got[t]:
            xe, ie, se = expected[j]
            assert iters == ie and status == se, (j, iters, ie)
            assert np.array_equal(x, xe), j
