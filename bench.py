"""Benchmark: QTW CG time to a 1e-12 relative residual on the 3D 7-point
Poisson problem 128^3 (n = 2,097,152, nnz = 14,581,760), one MI355X.

One step = one complete CG solve (x0 = 0, QTW arithmetic, tol 1e-12) with
the matrix, b and workspace already resident in HBM.  The JSON line adds:
  roofline      the dominant kernel (the CG-mode SpMV) measured live with
                HIP events around each of its launches during the timed
                steps; algorithmic bytes per launch
                12 nnz + 4 (n + 1) + 16 k n (k = 3 words);
  cpu_baseline  the CPU oracle on this host, timed on a bounded sample (a
                few CG iterations of the same solve), scaled to the solve's
                iteration count;
  extra         SpMV GB/s for every arithmetic (MALL flushed between
                repetitions), time to solution of every arithmetic, the
                QTW / DW time ratio, per-kernel times.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
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
WORDS = {"fp64": 1, "dw": 2, "qdw": 2, "tw": 3, "qtw": 3}


def spmv_bytes(n, nnz, k):
    return 12 * nnz + 4 * (n + 1) + 16 * k * n


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the per-arithmetic extras")
    ap.add_argument("--cpu-iters", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_13536_amd import mw, problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t = time.time()
    A, b, _ = P.case_poisson3d(args.nx)
    log("problem: 3D Poisson %d^3 n=%d nnz=%d (%.1fs)" % (args.nx, A.n, A.nnz, time.time() - t))
    Ad = mw.DeviceCSR.from_host(A, dev)
    bd = torch.as_tensor(b, device=dev)
    arith = "qtw"
    k = WORDS[arith]
    tol = 1e-12
    maxit = 10 * A.n
    ws = mw.cg_workspace(arith, Ad)
    x = torch.zeros((k, A.n), dtype=torch.float64, device=dev)

    for _ in range(args.warmup):
        x.zero_()
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws)
        log("warmup solve: %s" % info)
    torch.cuda.synchronize()

    prof = mw.CgProf()
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        _, info = mw.cg_solve(arith, Ad, bd, x=x, tol=tol, maxit=maxit, workspace=ws, prof=prof)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    iters = infos[-1]["iters"]
    assert all(i["status"] == "ok" for i in infos), infos
    log("timed: %.2f ms/solve, %d iterations, device %.2f ms" % (ms_per_step, iters, 1e3 * infos[-1]["seconds"]))

    pd = prof.as_dict()
    sp_us = pd["spmv"]["avg_us"]
    sp_bytes = spmv_bytes(A.n, A.nnz, k)
    achieved = sp_bytes / (sp_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "mw_spmv_kernel<QTW, CG mode>", "bytes_per_launch": sp_bytes,
                "avg_launch_us": round(sp_us, 2), "launches": pd["spmv"]["launches"]}

    extra = {"iterations": iters, "device_seconds": infos[-1]["seconds"],
             "per_iteration_us": 1e3 * ms_per_step / max(iters, 1),
             "kernel_avg_us": {c: (round(v["avg_us"], 2) if v["avg_us"] else None) for c, v in pd.items()}}

    if not args.quick:
        # SpMV bandwidth for every arithmetic, MALL flushed between repetitions
        flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        gbs = {}
        for ar in WORDS:
            kk = WORDS[ar]
            xv = torch.rand((kk, A.n), dtype=torch.float64, device=dev)
            yv = torch.empty_like(xv)
            ts = []
            for rep in range(25):
                flush.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mw.spmv(ar, Ad, xv, yv)
                e1.record()
                torch.cuda.synchronize()
                if rep >= 3:
                    ts.append(e0.elapsed_time(e1))
            med = statistics.median(ts)
            gbs[ar] = round(spmv_bytes(A.n, A.nnz, kk) / (med * 1e-3) / 1e9, 1)
        del flush
        extra["spmv_GBps_flushed"] = gbs
        log("SpMV GB/s: %s" % gbs)
        # time to solution of every arithmetic (one solve each, after warm-up)
        tts = {}
        for ar in WORDS:
            kk = WORDS[ar]
            wsa = mw.cg_workspace(ar, Ad)
            xa = torch.zeros((kk, A.n), dtype=torch.float64, device=dev)
            mw.cg_solve(ar, Ad, bd, x=xa, tol=tol, maxit=50, workspace=wsa)
            xa.zero_()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, ia = mw.cg_solve(ar, Ad, bd, x=xa, tol=tol, maxit=maxit, workspace=wsa)
            torch.cuda.synchronize()
            tts[ar] = {"seconds": round(time.perf_counter() - s0, 5), "iters": ia["iters"], "status": ia["status"]}
            log("%s: %s" % (ar, tts[ar]))
        extra["time_to_solution"] = tts
        extra["qtw_over_dw"] = round(tts["qtw"]["seconds"] / tts["dw"]["seconds"], 3)

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
               "sample": "%d QTW CG iterations of the same 128^3 solve (difference of maxit=%d and maxit=2 runs); "
                         "per-iteration time %.3f s x the GPU solve's %d iterations plus setup (extrapolated)"
                         % (ci, 2 + ci, per_iter, iters)}
        log("cpu baseline: %s" % cpu)

    out = {"metric": METRIC, "value": round(ms_per_step / 1e3, 5), "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "3D 7-point Poisson %d^3 (n=%d, nnz=%d), FP64 CSR int32, x_true~U[-1,1] seed 2, "
                                  "b=A x_true; QTW CG from x0=0 to ||r||/||b||<1e-12" % (args.nx, A.n, A.nnz),
                      "arith": arith, "tol": tol, "n": A.n, "nnz": A.nnz},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
