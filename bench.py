"""Benchmark: QTW CG time to a 1e-12 relative residual on the 3D 7-point
Poisson problem 128^3 (n = 2,097,152, nnz = 14,581,760), one MI355X.

One step = one complete CG solve (x0 = 0, QTW arithmetic, tol 1e-12) with
the matrix, its SpMV plan, b and workspace already resident in HBM, run the
way a caller solving repeatedly with one matrix runs it (plan built once in
the set-up, iteration chunks replayed from a captured hipGraph).  The JSON line
adds:
  roofline      the dominant kernel (the CG-mode SpMV): HIP events around
                each of its launches on the solver's stream, over solves
                run right after the timed steps with the same kernels
                launched directly (events recorded inside a replayed graph
                cannot be read back); algorithmic bytes per launch
                12 nnz + 4 (n + 1) + 16 k n (k = 3 words), the CSR
                definition; the plan's diagonal-slot slices stream fewer
                (format_bytes_per_launch, no column indices);
  cpu_baseline  the CPU oracle on this host, timed on a bounded sample (a
                few CG iterations of the same solve), scaled to the solve's
                iteration count;
  extra         SpMV GB/s for every arithmetic (MALL flushed between
                repetitions), time to solution of every arithmetic, the
                QTW / DW time ratio, per-kernel times, the batched and
                adjoint workloads and the two together (gradients of the
                512 systems), the ill-conditioned banded matrix,
                normalisation frequencies, tolerances beyond FP64 with
                true residuals, error norms against an exact integer
                solution, and one GPU's share of an 8-way split.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
One workload alone (its own JSON line, for profiling): --table1-only,
--batched-only, --illcond-only, --adjoint-only, --batched-adjoint-only.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QTW CG time-to-1e-12 residual & SpMV HBM GB/s; batched/adjoint vs plain"
HBM_PEAK_GBS = 8000.0
# planes of a vector element (the mixed types MXDW / MXQTW keep FP64 vectors)
WORDS = {"fp64": 1, "dw": 2, "qdw": 2, "tw": 3, "qtw": 3, "qtwe": 3, "qw": 4, "qqw": 4, "mxdw": 1, "mxqtw": 1}
ARITH_CODE = {"fp64": 0, "dw": 1, "qdw": 2, "tw": 3, "qtw": 4, "qtwe": 5, "qw": 6, "qqw": 7, "mxdw": 8, "mxqtw": 9}


def spmv_bytes(n, nnz, k):
    return 12 * nnz + 4 * (n + 1) + 16 * k * n


def kernel_source_hash():
    """Hash of the sources the SpMV kernel is compiled from (its file, the
    headers it includes, the ABI header): stored traffic figures are
    reported only while the kernel is the one that was profiled."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_13536_amd", "csrc")
    for f in ("mw_arith.hpp", "mw_common.hpp", "mw_blas.hpp", "mw_blas.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "mw.h"), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when absent
    or taken on other kernel sources."""
    p = os.path.join(ROOT, "profiles", "cg_qtw_poisson3d_128_traffic.json")
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return round(k["traffic_bytes"]) if k else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_ceiling(torch, dev, nbytes=1 << 30, reps=10):
    """Device copy bandwidth: bytes read + written over the median time of
    `reps` copies of a 1 GiB buffer (four times the Infinity Cache), the
    better of the runtime's copy (b.copy_(a)) and an elementwise kernel
    (b = a * 1)."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    best = 0.0
    for op in (lambda: b.copy_(a), lambda: torch.mul(a, 1.0, out=b)):
        ts = []
        for rep in range(reps + 2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            op()
            e1.record()
            torch.cuda.synchronize()
            if rep >= 2:
                ts.append(e0.elapsed_time(e1))
        best = max(best, 2 * nbytes / (statistics.median(ts) * 1e-3) / 1e9)
    del a, b
    return best


def bench_batched(mw, P, torch, dev, nsys=512, tune=True, loop=True):
    """512 uneven SPD systems (Poisson 2D/3D and circulant Laplacians, n in
    [1024, 65536]): one batched solve vs a loop of single solves, QTW and
    DW, tol 1e-12 (loop=False: the batched solves alone, for profiling);
    then the batched solve alone in the mixed types MXDW and MXQTW."""
    import numpy as np
    B = P.batch_systems(nsys=nsys)
    Ad = mw.DeviceCSR.from_host(B.A, dev)
    bd = torch.as_tensor(B.b, device=dev)
    subs = [B.system(s) for s in range(B.nsys)]
    devs = [(mw.DeviceCSR.from_host(A, dev), torch.as_tensor(b, device=dev)) for A, b in subs]
    out = {"workload": "%d systems, n=%d, nnz=%d" % (B.nsys, B.A.n, B.A.nnz)}
    for ar in ("qtw", "dw"):
        k = WORDS[ar]
        x = torch.zeros((k, B.A.n), dtype=torch.float64, device=dev)
        shape = mw.cg_batched_tune(ar, Ad, B.sys_row_off, bd, iters=16) if tune else None
        mw.cg_solve_batched(ar, Ad, B.sys_row_off, bd, x=x, tol=1e-12, maxit=100)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, iters, status, rel, info = mw.cg_solve_batched(ar, Ad, B.sys_row_off, bd, x=x, tol=1e-12)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out[ar] = {"batched_s": round(tb, 4), "tuned_grid": shape["spmv_grid"] if shape else None,
                   "max_iters": int(iters.max()), "mean_iters": round(float(iters.mean()), 1),
                   "all_converged": bool((status == 0).all())}
        if loop:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = []
            for (A, b) in devs:
                its.append(mw.cg_solve(ar, A, b, tol=1e-12)[1]["iters"])
            torch.cuda.synchronize()
            tl = time.perf_counter() - t0
            its = np.array(its)
            out[ar].update({"loop_s": round(tl, 4), "speedup": round(tl / tb, 2),
                            "iters_within_2pct_of_loop":
                                float(np.mean(np.abs(its - iters) <= np.maximum(1, 0.02 * its)))})
        log("batched %s: %s" % (ar, out[ar]))
    # the mixed types (FP64 vectors, rows and dots in DW / QTW), batched solve only
    for ar in ("mxdw", "mxqtw"):
        x = torch.zeros((WORDS[ar], B.A.n), dtype=torch.float64, device=dev)
        shape = mw.cg_batched_tune(ar, Ad, B.sys_row_off, bd, iters=16) if tune else None
        mw.cg_solve_batched(ar, Ad, B.sys_row_off, bd, x=x, tol=1e-12, maxit=100)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, iters, status, rel, info = mw.cg_solve_batched(ar, Ad, B.sys_row_off, bd, x=x, tol=1e-12)
        torch.cuda.synchronize()
        out[ar] = {"batched_s": round(time.perf_counter() - t0, 4), "tuned_grid": shape["spmv_grid"] if shape else None,
                   "max_iters": int(iters.max()), "mean_iters": round(float(iters.mean()), 1),
                   "all_converged": bool((status == 0).all())}
        log("batched %s: %s" % (ar, out[ar]))
    return out


def residual_levels(hist, every):
    """From a per-iteration relative-residual history: the first iteration
    below each power of ten reached, the smallest residual and where it
    occurred, and the history sampled every `every` iterations."""
    import numpy as np
    h = np.asarray(hist, dtype=np.float64)
    out = {"min_rel_res": None, "min_at": None, "first_below": {}, "every": every, "sampled": []}
    if h.size == 0:
        return out
    fin = np.where(np.isfinite(h), h, np.inf)
    i = int(np.argmin(fin))
    out["min_rel_res"], out["min_at"] = float(fin[i]), i + 1
    for e in range(-1, -21, -1):
        below = np.nonzero(fin < 10.0 ** e)[0]
        if below.size == 0:
            break
        out["first_below"]["1e%d" % e] = int(below[0]) + 1
    out["sampled"] = [float("%.4g" % v) for v in h[every - 1::every]]
    return out


def bench_illcond(mw, P, torch, dev, maxit=20000, hist_every=0):
    """Ill-conditioned banded SPD (n = 2^20, 27 nnz/row, D A D scaled):
    planned SpMV GB/s (Infinity Cache read-flushed) and a CG run of at most
    `maxit` iterations toward 1e-10 in FP64, DW and QTW (relative residual
    reached, time per iteration); with hist_every > 0 also the residual
    history (first iteration below each power of ten, the lowest level and
    samples every hist_every iterations); Jacobi-preconditioned CG to 1e-10
    and 1e-20."""
    A, b, _ = P.case_banded_illcond()
    Ad = mw.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(b, device=dev)
    plan = mw.Plan(Ad)
    flush = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    out = {"workload": "banded SPD offsets +-1..13, D A D (D_ii = 10^U(-3,3)), n=%d, nnz=%d, tol 1e-10, "
                       "at most %d iterations" % (A.n, A.nnz, maxit)}
    for ar in ("fp64", "dw", "qtw", "mxdw", "mxqtw"):
        kk = WORDS[ar]
        xv = torch.rand((kk, A.n), dtype=torch.float64, device=dev)
        yv = torch.empty_like(xv)
        ts = []
        for rep in range(8):
            sink.copy_(flush.sum().reshape(1))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mw.spmv_planned(ar, plan, xv, yv)
            e1.record()
            torch.cuda.synchronize()
            if rep >= 2:
                ts.append(e0.elapsed_time(e1))
        gbs = spmv_bytes(A.n, A.nnz, kk) / (statistics.median(ts) * 1e-3) / 1e9
        x = torch.zeros((kk, A.n), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = mw.cg_solve(ar, Ad, bd, x=x, tol=1e-10, maxit=maxit, history=hist_every > 0)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[ar] = {"spmv_GBps_planned_flushed": round(gbs, 1), "iters": info["iters"], "status": info["status"],
                   "rel_res": info["rel_res"], "seconds": round(sec, 3),
                   "per_iteration_us": round(1e6 * sec / max(info["iters"], 1), 1)}
        if hist_every > 0:
            out[ar]["history"] = residual_levels(info["history"], hist_every)
            out[ar]["true_rel_res"] = true_rel_residual(mw, torch, Ad, bd, x)
            log("ill-conditioned %s, %d iterations: %s, rel. residual %.3e, lowest %.3e at %d, %s"
                % (ar, info["iters"], info["status"], info["rel_res"], out[ar]["history"]["min_rel_res"],
                   out[ar]["history"]["min_at"], out[ar]["history"]["first_below"]))
        # Jacobi-preconditioned CG (an extension; it removes the D A D
        # scaling): iterations, time and the exactly formed true residual
        # (the mixed types keep z = D r in FP64 as well)
        for ptol in (1e-10, 1e-20):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, pinfo = mw.cg_solve(ar, Ad, bd, x=x, tol=ptol, maxit=maxit, precond="jacobi")
            torch.cuda.synchronize()
            out[ar]["jacobi_tol_%g" % ptol] = {"status": pinfo["status"], "iters": pinfo["iters"],
                                               "seconds": round(time.perf_counter() - t0, 5),
                                               "true_rel_res": true_rel_residual(mw, torch, Ad, bd, x)}
        log("ill-conditioned %s: %s" % (ar, out[ar]))
    return out


def bench_normalisation(mw, torch, Ad, bd, n, maxit=2000):
    """3D Poisson 128^3, QDW, QTW and QQW, tol 1e-12: r normalised every K-th
    iteration (K = 1 is the paper's placement, 0 never), and the placement
    variant that normalises p with r ("K=..+p"): status, iterations, time;
    for the variant also the true residual at tol 1e-30 (QDW) / 1e-44 (QTW,
    QQW) against K = 1's; and QTWE, VecSum3 after every operation (the other
    end of the placement range; for QDW that placement is DW itself)."""
    out = {"workload": "3D Poisson 128^3, tol 1e-12, at most %d iterations" % maxit}
    for ar in ("qdw", "qtw", "qqw"):
        x = torch.zeros((WORDS[ar], n), dtype=torch.float64, device=bd.device)
        row = {}
        for K, npz in ((1, False), (2, False), (4, False), (8, False), (0, False),
                       (2, True), (8, True), (32, True), (64, True)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = mw.cg_solve(ar, Ad, bd, x=x, tol=1e-12, maxit=maxit, normalize=K, normalize_p=npz)
            torch.cuda.synchronize()
            row["K=%d%s" % (K, "+p" if npz else "")] = {
                "status": info["status"], "iters": info["iters"], "rel_res": info["rel_res"],
                "seconds": round(time.perf_counter() - t0, 4)}
        tight = 1e-30 if WORDS[ar] == 2 else 1e-44
        for K, npz in ((1, False), (8, True), (64, True)):
            x.zero_()
            _, info = mw.cg_solve(ar, Ad, bd, x=x, tol=tight, maxit=3 * maxit, normalize=K, normalize_p=npz)
            row["tol_%g_K=%d%s" % (tight, K, "+p" if npz else "")] = {
                "status": info["status"], "iters": info["iters"], "true_rel_res": true_rel_residual(mw, torch, Ad, bd, x)}
        out[ar] = row
        log("normalisation %s: %s" % (ar, row))
    x = torch.zeros((3, n), dtype=torch.float64, device=bd.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = mw.cg_solve("qtwe", Ad, bd, x=x, tol=1e-12, maxit=maxit)
    torch.cuda.synchronize()
    out["qtwe_every_operation"] = {"status": info["status"], "iters": info["iters"], "rel_res": info["rel_res"],
                                   "seconds": round(time.perf_counter() - t0, 4)}
    log("normalisation qtwe (every operation): %s" % out["qtwe_every_operation"])
    return out


def true_rel_residual(mw, torch, Ad, bd, x):
    """||b - A x|| / ||b|| for a solution in any arithmetic, with the product,
    the difference and the dots formed in QW (about 64 significant digits),
    so residuals far below FP64 resolution are resolved."""
    n = x.shape[1]
    x4 = torch.zeros((4, n), dtype=torch.float64, device=bd.device)
    x4[:x.shape[0]] = x
    b4 = torch.zeros_like(x4)
    b4[0] = bd
    y = mw.spmv("qw", Ad, x4)
    r = mw.elementwise("qw", "add", b4, mw.elementwise("qw", "neg", y))
    rr = float(mw.dot("qw", r, r).sum().item())
    bb = float(mw.dot("qw", b4, b4).sum().item())
    return (max(rr, 0.0) / bb) ** 0.5


def bench_tolerances(mw, torch, Ad, bd, n, maxit=4000):
    """3D Poisson 128^3 at tolerances beyond FP64 (1e-16, 1e-24, 1e-32, 1e-48,
    and 1e-60 for the 4-word types), every arithmetic, at most `maxit`
    iterations: status, iterations, time, the recursive and the true
    relative residual (true_rel_residual), and the recursive
    relative-residual history of the 1e-32 runs every 50 iterations."""
    out = {"workload": "3D Poisson 128^3, at most %d iterations" % maxit}
    for ar in WORDS:
        x = torch.zeros((WORDS[ar], n), dtype=torch.float64, device=bd.device)
        row = {}
        for tol in (1e-16, 1e-24, 1e-32, 1e-48) + ((1e-60,) if WORDS[ar] == 4 else ()):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = mw.cg_solve(ar, Ad, bd, x=x, tol=tol, maxit=maxit, history=(tol == 1e-32))
            torch.cuda.synchronize()
            row["tol_%g" % tol] = {"status": info["status"], "iters": info["iters"], "rel_res": info["rel_res"],
                                   "seconds": round(time.perf_counter() - t0, 4),
                                   "true_rel_res": true_rel_residual(mw, torch, Ad, bd, x)}
            if tol == 1e-32:
                h = info["history"]
                row["history_every_50"] = [float("%.3e" % v) for v in h[49::50]]
        out[ar] = row
        log("tolerances %s: %s" % (ar, {k: v for k, v in row.items() if k != "history_every_50"}))
    return out


def bench_error_history(mw, P, torch, dev, nx=128, seed=6,
                        checkpoints=(100, 200, 400, 600, 800, 1000, 1200, 1600, 2000, 2400)):
    """Error norms against an exact solution: 3D Poisson nx^3 with an
    integer solution x* in [-8, 8] (seed `seed`), so b = A x* is exact in
    FP64.  For every arithmetic and every checkpoint m: ||x_m - x*|| / ||x*||
    and the true relative residual of the m-th CG iterate from x_0 = 0.  The
    m-th iterate is the result of a solve stopped after m iterations (tol 0;
    the solver is deterministic for a fixed launch shape, so it is the m-th
    iterate of the full solve).  x_m - x* is formed in QW before it is
    rounded to FP64."""
    A = P.poisson3d(nx)
    xs = P.integer_vector(A.n, seed)
    Ad = mw.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(A.matvec(xs), device=dev)
    xs4 = torch.zeros((4, A.n), dtype=torch.float64, device=dev)
    xs4[0] = torch.as_tensor(xs, device=dev)
    nxs = float(torch.linalg.vector_norm(xs4[0]).item())
    plan = mw.Plan(Ad)
    out = {"workload": "3D Poisson %d^3, x* integer in [-8, 8] (seed %d), b = A x* exact" % (nx, seed),
           "checkpoints": list(checkpoints)}
    for ar in WORDS:
        k = WORDS[ar]
        ws = mw.cg_workspace(ar, Ad)
        x = torch.zeros((k, A.n), dtype=torch.float64, device=dev)
        err, res = [], []
        for m in checkpoints:
            x.zero_()
            mw.cg_solve(ar, Ad, bd, x=x, tol=0.0, maxit=m, workspace=ws, plan=plan)
            x4 = torch.zeros_like(xs4)
            x4[:k] = x
            d = mw.elementwise("qw", "add", x4, mw.elementwise("qw", "neg", xs4))
            err.append(float("%.3e" % (float(torch.linalg.vector_norm(d[0]).item()) / nxs)))
            res.append(float("%.3e" % true_rel_residual(mw, torch, Ad, bd, x)))
        out[ar] = {"rel_error": err, "true_rel_res": res}
        log("error history %s: %s" % (ar, out[ar]))
    return out


def bench_table1(mw, P, torch, dev, iters=100):
    """Per-iteration CG time of every arithmetic on banded stand-ins of the
    paper's Table I matrices (same n and nonzeros per row; P.TABLE1), and
    the ratio to FP64 -- the quantity of the paper's relative-time figure
    (Sec. V-B), measured here on one MI355X.  `iters` iterations (tol 0),
    after one short warm-up solve; the SpMV plan is the one the solver
    builds for itself (vector rows for the matrices of at most 2^18 rows,
    with the lanes per row of its rule; else SELL-64), built once per
    matrix and arithmetic."""
    import numpy as np
    out = {"iterations": iters}
    for name, _, _ in P.TABLE1:
        A = P.table1_standin(name)
        Ad = mw.DeviceCSR.from_host(A, dev)
        b = torch.as_tensor(A.matvec(np.random.default_rng(7).uniform(-1, 1, A.n)), device=dev)
        row = {"n": A.n, "nnz": A.nnz, "plan": {}}
        for ar in WORDS:
            plan = mw.Plan(Ad, solver=ar)
            row["plan"][ar] = "rows/%d" % plan.lanes if plan.format == "csrvec" else plan.format
            ws = mw.cg_workspace(ar, Ad)
            x = torch.zeros((WORDS[ar], A.n), dtype=torch.float64, device=dev)
            mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=4, workspace=ws, plan=plan)
            best = None
            for _ in range(2):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=iters, workspace=ws, plan=plan)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                best = t if best is None else min(best, t)
            row[ar] = round(1e6 * best / max(info["iters"], 1), 1)
        row["over_fp64"] = {ar: round(row[ar] / row["fp64"], 2) for ar in WORDS if ar != "fp64"}
        row["qtw_over_dw"] = round(row["qtw"] / row["dw"], 2)
        # for comparison: FP64 and QTW with the SELL-64 plan (one lane per row)
        splan = mw.Plan(Ad)
        for ar in ("fp64", "qtw"):
            ws = mw.cg_workspace(ar, Ad)
            x = torch.zeros((WORDS[ar], A.n), dtype=torch.float64, device=dev)
            mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=4, workspace=ws, plan=splan)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=iters, workspace=ws, plan=splan)
            torch.cuda.synchronize()
            row["%s_%s_us" % (splan.format, ar)] = round(1e6 * (time.perf_counter() - t0) / max(info["iters"], 1), 1)
        out[name] = row
        log("table I stand-in %s: %s" % (name, row))
        del Ad, plan, splan
    return out


def bench_shard(mw, P, torch, dev, parts=8, iters=200):
    """One GPU's share of the 128^3 problem split into `parts` z-slabs: the
    rows of 128^3 / parts planes plus one halo plane on each side (the
    rows a shard's SpMV gathers from its neighbours), as a 128 x 128 x
    (128 / parts + 2) Poisson matrix.  Planned SpMV GB/s (Infinity Cache
    read-flushed) and the time of a CG iteration (tol 0, `iters`
    iterations) per arithmetic, to compare with the full problem."""
    import numpy as np
    nz = 128 // parts + 2
    A = P.poisson3d(128, 128, nz)
    Ad = mw.DeviceCSR.from_host(A, dev)
    b = torch.as_tensor(A.matvec(np.random.default_rng(2).uniform(-1, 1, A.n)), device=dev)
    plan = mw.Plan(Ad)
    flush = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    out = {"workload": "3D Poisson 128 x 128 x %d (%d-way z-slab share + 2 halo planes), n=%d, nnz=%d"
                       % (nz, parts, A.n, A.nnz)}
    for ar in ("fp64", "dw", "qtw"):
        kk = WORDS[ar]
        xv = torch.rand((kk, A.n), dtype=torch.float64, device=dev)
        yv = torch.empty_like(xv)
        ts = []
        for rep in range(10):
            sink.copy_(flush.sum().reshape(1))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mw.spmv_planned(ar, plan, xv, yv)
            e1.record()
            torch.cuda.synchronize()
            if rep >= 2:
                ts.append(e0.elapsed_time(e1))
        gbs = spmv_bytes(A.n, A.nnz, kk) / (statistics.median(ts) * 1e-3) / 1e9
        x = torch.zeros((kk, A.n), dtype=torch.float64, device=dev)
        mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=iters, plan=plan)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = mw.cg_solve(ar, Ad, b, x=x, tol=0.0, maxit=iters, plan=plan)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[ar] = {"spmv_GBps_planned_flushed": round(gbs, 1), "per_iteration_us": round(1e6 * sec / iters, 1)}
        log("shard %s: %s" % (ar, out[ar]))
    return out


def bench_adjoint(mw, P, torch, dev):
    """A(theta) = 3D Laplacian 100^3 + diag(theta), loss 0.5||x - x_t||^2,
    QTW: forward + adjoint solve (all 2n gradient entries) vs the cost of
    central finite differences (2 solves per coordinate)."""
    from paper_2510_13536_amd import adjoint
    Q = P.adjoint_problem(nx=100)
    Ad = mw.DeviceCSR.from_host(Q.lap, dev)
    lap_val = torch.as_tensor(Q.lap.val, device=dev)
    pos = torch.as_tensor(Q.diag_pos, device=dev)
    xt = torch.as_tensor(Q.x_target, device=dev)
    out = {"workload": "3D Laplacian 100^3 + diag(theta), n=%d, nnz=%d, QTW" % (Q.lap.n, Q.lap.nnz)}
    for tol in (1e-12, 1e-24):
        times = []
        for rep in range(2):
            theta = torch.as_tensor(Q.theta, device=dev).requires_grad_(True)
            b = torch.as_tensor(Q.b, device=dev).requires_grad_(True)
            info = {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = adjoint.cg_solve(Ad, lap_val.index_add(0, pos, theta), b, arith="qtw", tol=tol, info=info)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            (0.5 * ((x - xt) ** 2).sum()).backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1, info["forward"]["iters"], info["adjoint"]["iters"]))
        fwd, bwd, itf, itb = times[-1]
        out["tol_%g" % tol] = {"forward_s": round(fwd, 4), "backward_s": round(bwd, 4),
                               "backward_over_forward": round(bwd / fwd, 3), "forward_iters": itf,
                               "adjoint_iters": itb, "fd_s_per_coordinate": round(2 * fwd, 4),
                               "fd_s_for_all_2n_coordinates": round(2 * fwd * 2 * Q.lap.n, 1)}
        log("adjoint tol %g: %s" % (tol, out["tol_%g" % tol]))
    return out


def bench_batched_adjoint(mw, P, torch, dev, nsys=512):
    """The 512-system batch with theta ~ U[0.01, 1] (seed 6) added to its
    diagonal, loss 0.5 ||x - x_target||^2 (x_target ~ N(0, 1), seed 66), QTW
    to 1e-12: all systems' theta and b gradients from one batched forward
    and one batched adjoint solve, against a loop of single-system adjoints."""
    import numpy as np
    from paper_2510_13536_amd import adjoint
    B = P.batch_systems(nsys=nsys)
    theta0 = np.random.default_rng(6).uniform(0.01, 1.0, B.A.n)
    xt0 = np.random.default_rng(66).standard_normal(B.A.n)
    Ad = mw.DeviceCSR.from_host(B.A, dev)
    pos = torch.as_tensor(P.diagonal_positions(B.A), device=dev)
    lap_val = torch.as_tensor(B.A.val, device=dev)
    xt = torch.as_tensor(xt0, device=dev)
    out = {"workload": "%d systems, n=%d, nnz=%d, + diag(theta), QTW, tol 1e-12" % (B.nsys, B.A.n, B.A.nnz)}
    times = []
    for rep in range(2):
        theta = torch.as_tensor(theta0, device=dev).requires_grad_(True)
        b = torch.as_tensor(B.b, device=dev).requires_grad_(True)
        info = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = adjoint.cg_solve_batched(Ad, lap_val.index_add(0, pos, theta), B.sys_row_off, b, arith="qtw", tol=1e-12,
                                     info=info)
        (0.5 * ((x - xt) ** 2).sum()).backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    out["batched_s"] = round(times[-1], 4)
    out["forward_iters_max"] = int(info["forward"]["iters"].max())
    out["adjoint_iters_max"] = int(info["adjoint"]["iters"].max())
    # the loop: one single-system differentiable solve per system
    subs = []
    for s in range(B.nsys):
        lo, hi = int(B.sys_row_off[s]), int(B.sys_row_off[s + 1])
        A, bs = B.system(s)
        subs.append((mw.DeviceCSR.from_host(A, dev), torch.as_tensor(A.val, device=dev),
                     torch.as_tensor(P.diagonal_positions(A), device=dev), lo, hi, bs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for As, vals, ps, lo, hi, bs in subs:
        th = torch.as_tensor(theta0[lo:hi], device=dev).requires_grad_(True)
        bb = torch.as_tensor(bs, device=dev).requires_grad_(True)
        x = adjoint.cg_solve(As, vals.index_add(0, ps, th), bb, arith="qtw", tol=1e-12)
        (0.5 * ((x - xt[lo:hi]) ** 2).sum()).backward()
    torch.cuda.synchronize()
    out["loop_s"] = round(time.perf_counter() - t0, 4)
    out["speedup"] = round(out["loop_s"] / out["batched_s"], 2)
    log("batched adjoint: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the per-arithmetic extras")
    ap.add_argument("--arith", default="qtw", choices=sorted(WORDS),
                    help="arithmetic of the timed solve (the headline metric is QTW)")
    ap.add_argument("--cpu-iters", type=int, default=16)
    ap.add_argument("--prof-steps", type=int, default=2, help="event-timed solves for the roofline")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape tuner (built-in shapes)")
    ap.add_argument("--table1", action="store_true",
                    help="also time iterations on banded stand-ins of the paper's Table I matrices")
    ap.add_argument("--table1-only", action="store_true",
                    help="run only the Table I stand-ins (per-iteration time of every arithmetic) and print their line")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 512-system batched comparison (for profiling that path) and print its line")
    ap.add_argument("--no-loop", action="store_true",
                    help="with --batched-only: skip the loop of single solves (for profiling the batched one)")
    ap.add_argument("--batched-adjoint-only", action="store_true",
                    help="run only the batched differentiable solve on the 512-system batch and print its line")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint workload (forward + adjoint QTW solves) and print its line")
    ap.add_argument("--illcond-only", action="store_true",
                    help="run only the ill-conditioned banded workload and print its line")
    ap.add_argument("--illcond-maxit", type=int, default=20000,
                    help="iteration limit of the ill-conditioned CG runs")
    ap.add_argument("--illcond-hist", type=int, default=0,
                    help="record the ill-conditioned runs' residual history, sampled every N iterations")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_13536_amd import mw, problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calib_copy:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.table1_only:
        t1 = bench_table1(mw, P, torch, dev)
        print(json.dumps({"metric": "CG time per iteration on banded stand-ins of the paper's Table I matrices",
                          "value": t1["nd24k"]["qtw"], "unit": "us", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": "Table I stand-ins"},
                          "extra": {"table1_standins": t1}}), flush=True)
        return
    if args.batched_only:
        bt = bench_batched(mw, P, torch, dev, tune=not args.no_tune, loop=not args.no_loop)
        print(json.dumps({"metric": "batched QTW CG time-to-1e-12 (512 systems, one lockstep solve)",
                          "value": bt["qtw"]["batched_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": bt["workload"]},
                          "extra": {"batched": bt}}), flush=True)
        return
    if args.batched_adjoint_only:
        ba = bench_batched_adjoint(mw, P, torch, dev)
        print(json.dumps({"metric": "batched adjoint gradients (512 systems + diag theta, QTW, tol 1e-12)",
                          "value": ba["batched_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": ba["workload"]},
                          "extra": {"batched_adjoint": ba}}), flush=True)
        return
    if args.adjoint_only:
        ad = bench_adjoint(mw, P, torch, dev)
        print(json.dumps({"metric": "adjoint gradient (forward + adjoint QTW solve), tol 1e-12",
                          "value": round(ad["tol_1e-12"]["forward_s"] + ad["tol_1e-12"]["backward_s"], 4),
                          "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": ad["workload"]}, "extra": {"adjoint": ad}}), flush=True)
        return
    if args.illcond_only:
        ic = bench_illcond(mw, P, torch, dev, maxit=args.illcond_maxit, hist_every=args.illcond_hist)
        print(json.dumps({"metric": "ill-conditioned banded CG (n=2^20, 27 nnz/row, D A D), tol 1e-10",
                          "value": ic["qtw"]["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": ic["workload"]},
                          "extra": {"illcond": ic}}), flush=True)
        return
    t = time.time()
    A, b, _ = P.case_poisson3d(args.nx)
    log("problem: 3D Poisson %d^3 n=%d nnz=%d (%.1fs)" % (args.nx, A.n, A.nnz, time.time() - t))
    Ad = mw.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(b, device=dev)
    arith = args.arith
    k = WORDS[arith]
    tol = 1e-12
    maxit = 10 * A.n
    ws = mw.cg_workspace(arith, Ad)
    x = torch.zeros((k, A.n), dtype=torch.float64, device=dev)

    # set-up, before the timed region: the SpMV plan of A (built once, as a
    # caller solving repeatedly with one matrix does) and the launch-shape
    # tuner's grids for this matrix
    splan = mw.Plan(Ad)
    tuned = None
    if not args.no_tune:
        t = time.time()
        tuned = mw.cg_tune(arith, Ad, bd, iters=32, workspace=ws)
        log("tuned shape: %s (%.2f s)" % (tuned, time.time() - t))
    for _ in range(args.warmup):
        x.zero_()
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws, plan=splan)
        log("warmup solve: %s" % info)
    torch.cuda.synchronize()

    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws, plan=splan)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    iters = infos[-1]["iters"]
    assert all(i["status"] == "ok" for i in infos), infos
    log("timed: %.2f ms/solve, %d iterations, device %.2f ms" % (ms_per_step, iters, 1e3 * infos[-1]["seconds"]))

    # kernel durations: the same solve with HIP events around every SpMV
    prof = mw.CgProf.of("spmv")
    pinfos = []
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(args.prof_steps):
        x.zero_()
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws, prof=prof, plan=splan)
        pinfos.append(info)
    torch.cuda.synchronize()
    prof_ms = 1e3 * (time.perf_counter() - p0) / max(args.prof_steps, 1)
    assert all(i["status"] == "ok" and i["iters"] == iters for i in pinfos), pinfos

    pd = prof.as_dict()
    sp_us = pd["spmv"]["avg_us"]
    sp_bytes = spmv_bytes(A.n, A.nnz, k)
    achieved = sp_bytes / (sp_us * 1e-6) / 1e9
    # what the planned SpMV actually streams: when every slice is stored as
    # diagonal slots, 8 bytes per stored value, 12 per slot (offset + lane
    # mask), 4 per slice pointer, 16 k per row (own p read, q written)
    plan = splan
    fmt_bytes = None
    if plan.format == "sell64" and plan.ndiag == plan.c.nslices:
        fmt_bytes = 8 * plan.stored + 12 * (plan.stored // 64) + 4 * (plan.c.nslices + 1) + 16 * k * A.n
    plan_info = {"format": plan.format, "nslices": int(plan.c.nslices), "diagonal_slices": plan.ndiag,
                 "stored_entries": plan.stored}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic("mw_sell_spmv_kernel<%d, 1>" % ARITH_CODE[arith]),
                "kernel": "mw_sell_spmv_kernel<%s, CG mode>" % arith.upper(), "bytes_per_launch": sp_bytes,
                "avg_launch_us": round(sp_us, 2), "launches": pd["spmv"]["launches"],
                "format_bytes_per_launch": fmt_bytes,
                "format_GBps": round(fmt_bytes / (sp_us * 1e-6) / 1e9, 1) if fmt_bytes else None,
                "plan": plan_info,
                "timing": "HIP events around each SpMV launch on the solver stream, %d event-timed solves "
                          "(direct launches, %.2f ms/solve) right after the timed steps" % (args.prof_steps, prof_ms)}
    # three byte counts for the same launch time: `frac` uses the CSR
    # definition's algorithmic bytes (the per-unit figure every arithmetic
    # and plan shares); the diagonal-slot plan streams fewer (no column
    # indices: format bytes), and the counters give what HBM really moved
    roofline["frac_basis"] = "CSR algorithmic bytes 12 nnz + 4 (n + 1) + 16 k n per launch"
    if fmt_bytes:
        roofline["format_frac"] = round(fmt_bytes / (sp_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    if roofline["traffic"]:
        tg = roofline["traffic"] / (sp_us * 1e-6) / 1e9
        roofline["traffic_GBps"] = round(tg, 1)
        roofline["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
    # the same kernel against what a plain device copy reaches on this GPU
    cc = copy_ceiling(torch, dev)
    roofline["copy_GBps"] = round(cc, 1)
    roofline["frac_of_copy"] = round(achieved / cc, 4)
    log("copy ceiling %.1f GB/s; SpMV %.1f GB/s = %.3f of it" % (cc, achieved, achieved / cc))

    # one call as a caller without a prebuilt plan makes it: mw_cg_solve
    # builds the SpMV plan inside the call, in its workspace
    one = []
    for _ in range(3):
        x.zero_()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        _, oi = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws)
        torch.cuda.synchronize()
        one.append(time.perf_counter() - s0)
        assert oi["status"] == "ok" and oi["iters"] == iters, oi
    one_call = {"seconds": round(statistics.median(one), 5),
                "what": "median of 3 mw_cg_solve calls with no plan passed (SpMV plan built inside each call)"}
    log("one call with the plan built inside: %.2f ms" % (1e3 * one_call["seconds"]))

    extra = {"iterations": iters, "device_seconds": infos[-1]["seconds"], "one_call_with_plan_build": one_call,
             "launch_shape": mw.cg_shape(arith, A.n, A.nnz)[1], "tuned": tuned is not None,
             "per_iteration_us": 1e3 * ms_per_step / max(iters, 1),
             "event_timed_ms_per_step": round(prof_ms, 3)}
    # every kernel class event-timed, one more solve
    pall = mw.CgProf()
    x.zero_()
    mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws, prof=pall, plan=splan)
    extra["kernel_avg_us"] = {c: (round(v["avg_us"], 2) if v["avg_us"] else None) for c, v in pall.as_dict().items()}

    if not args.quick:
        # Standalone SpMV bandwidth for every arithmetic, planned (SELL-64)
        # and plain CSR.  Before each repetition the 256 MB Infinity Cache is
        # flushed by READING a 1 GiB buffer (a write flush would leave dirty
        # lines whose write-back lands inside the timed kernel).
        flush = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        sink = torch.zeros(1, dtype=torch.float64, device=dev)
        plan = mw.Plan(Ad)
        gbs, gbs_csr = {}, {}
        for ar in WORDS:
            kk = WORDS[ar]
            xv = torch.rand((kk, A.n), dtype=torch.float64, device=dev)
            yv = torch.empty_like(xv)
            for fn, dst in ((lambda: mw.spmv_planned(ar, plan, xv, yv), gbs), (lambda: mw.spmv(ar, Ad, xv, yv), gbs_csr)):
                ts = []
                for rep in range(15):
                    sink.copy_(flush.sum().reshape(1))
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    fn()
                    e1.record()
                    torch.cuda.synchronize()
                    if rep >= 3:
                        ts.append(e0.elapsed_time(e1))
                dst[ar] = round(spmv_bytes(A.n, A.nnz, kk) / (statistics.median(ts) * 1e-3) / 1e9, 1)
        del flush, plan
        extra["spmv_GBps_planned_flushed"] = gbs
        extra["spmv_GBps_csr_flushed"] = gbs_csr
        log("SpMV GB/s planned: %s  csr: %s" % (gbs, gbs_csr))
        # time to solution of every arithmetic: every arithmetic tuned and
        # warmed up first, then three rounds that each solve once in every
        # arithmetic (so a slow drift of the GPU's clocks over the run does
        # not favour the arithmetics measured first), best solve of each;
        # the same prebuilt plan throughout
        tts, state = {}, {}
        for ar in WORDS:
            wsa = mw.cg_workspace(ar, Ad)
            xa = torch.zeros((WORDS[ar], A.n), dtype=torch.float64, device=dev)
            if not args.no_tune:
                mw.cg_tune(ar, Ad, bd, iters=32, workspace=wsa)
            mw.cg_solve(ar, Ad, bd, x=xa, tol=tol, maxit=50, workspace=wsa, plan=splan)
            state[ar] = (wsa, xa)
        for _ in range(3):
            for ar in WORDS:
                wsa, xa = state[ar]
                xa.zero_()
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                _, ia = mw.cg_solve(ar, Ad, bd, x=xa, tol=tol, maxit=maxit, workspace=wsa, plan=splan)
                torch.cuda.synchronize()
                t_ar = time.perf_counter() - s0
                if ar not in tts or t_ar < tts[ar]["seconds"]:
                    tts[ar] = {"seconds": round(t_ar, 5), "iters": ia["iters"], "status": ia["status"],
                               "shape": mw.cg_shape(ar, A.n, A.nnz)[1]}
        for ar in WORDS:
            log("%s: %s" % (ar, tts[ar]))
        del state
        extra["time_to_solution"] = tts
        extra["qtw_over_dw"] = round(tts["qtw"]["seconds"] / tts["dw"]["seconds"], 3)

    if not args.quick:
        extra["batched"] = bench_batched(mw, P, torch, dev, tune=not args.no_tune)
        extra["adjoint"] = bench_adjoint(mw, P, torch, dev)
        extra["batched_adjoint"] = bench_batched_adjoint(mw, P, torch, dev)
        extra["illcond"] = bench_illcond(mw, P, torch, dev, maxit=args.illcond_maxit)
        extra["normalisation_every_K"] = bench_normalisation(mw, torch, Ad, bd, A.n)
        extra["tolerances"] = bench_tolerances(mw, torch, Ad, bd, A.n)
        extra["error_history"] = bench_error_history(mw, P, torch, dev)
        extra["shard_8way"] = bench_shard(mw, P, torch, dev)
    if args.table1:
        extra["table1_standins"] = bench_table1(mw, P, torch, dev)

    cpu = None
    if not args.no_cpu:
        import oracle as O
        ci = args.cpu_iters
        s0 = time.perf_counter()
        O.cg_solve(arith, A, b, tol=tol, maxit=2)
        s1 = time.perf_counter()
        O.cg_solve(arith, A, b, tol=tol, maxit=2 + ci)
        s2 = time.perf_counter()
        per_iter = ((s2 - s1) - (s1 - s0)) / ci
        setup = max((s1 - s0) - 2 * per_iter, 0.0)
        cpu = {"value": round(setup + per_iter * iters, 2), "unit": "s", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": "%d %s CG iterations of the same %d^3 solve (difference of maxit=%d and maxit=2 runs); "
                         "per-iteration time %.3f s x the GPU solve's %d iterations plus setup (extrapolated)"
                         % (ci, arith.upper(), args.nx, 2 + ci, per_iter, iters)}
        log("cpu baseline: %s" % cpu)
        # the same oracle on one thread (a few iterations)
        nthr = O.num_threads()
        O.set_num_threads(1)
        c1 = max(2, ci // 4)
        s0 = time.perf_counter()
        O.cg_solve(arith, A, b, tol=tol, maxit=1)
        s1 = time.perf_counter()
        O.cg_solve(arith, A, b, tol=tol, maxit=1 + c1)
        s2 = time.perf_counter()
        O.set_num_threads(nthr)
        per1 = ((s2 - s1) - (s1 - s0)) / c1
        extra["cpu_oracle_1_thread"] = {"s_per_iteration": round(per1, 3), "extrapolated_s": round(per1 * iters, 1),
                                        "sample": "%d %s CG iterations on one thread (difference of maxit=%d and "
                                                  "maxit=1 runs)" % (c1, arith.upper(), 1 + c1)}
        log("cpu oracle, 1 thread: %s" % extra["cpu_oracle_1_thread"])

    out = {"metric": METRIC, "value": round(ms_per_step / 1e3, 5), "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "3D 7-point Poisson %d^3 (n=%d, nnz=%d), FP64 CSR int32, x_true~U[-1,1] seed 2, "
                                  "b=A x_true; %s CG from x0=0 to ||r||/||b||<1e-12" % (args.nx, A.n, A.nnz, arith.upper()),
                      "arith": arith, "tol": tol, "n": A.n, "nnz": A.nnz},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
