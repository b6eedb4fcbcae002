"""Writes the oracle's results on the full-size workloads that the GPU
parity tests compare against, so that those tests need not rerun
multi-minute CPU solves on every GPU run.  Calls only the oracle (oracle/)
and the seeded generators (paper_2510_13536_amd/problems.py).

  c2_oracle_solves.json   3D Poisson 128^3 (x* ~ U[-1,1] seed 2, b = A x*),
                          CG from x0 = 0 to 1e-12 in FP64, DW, QDW, TW, QTW,
                          QW, QQW, QTWE and the mixed MXDW / MXQTW
                          (Alg. 1 with Sec. IV-C/IV-D): status, iterations,
                          recursive relative residual and the true relative
                          residual ||b - A x|| / ||b|| of the oracle's x,
                          formed exactly.
  c4_oracle_solves.json   the 512-system batch (seed 4): the four largest
                          systems and four of median size, CG from x0 = 0
                          to 1e-12 in DW and QTW, the same fields.
  c5_oracle_gradient.json the adjoint problem 100^3 + diag(theta): the QTW
                          forward solve x = A^-1 b and adjoint solve
                          A lam = fp64(x) - x_target to 1e-26, and the
                          gradients -fp64(lam_i x_i) (theta) and fp64(lam)
                          (b) at the 64 + 64 coordinates drawn with seed 5555
                          (theta first, then b), with their largest
                          magnitudes over all coordinates.

Usage: python tests/golden/make_fullsize_oracle.py [c2] [c4] [c5]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2510_13536_amd import problems as P  # noqa: E402


# the mixed types: FP64 vectors, SpMV rows and dots in their base arithmetic
MIXED = {"mxdw": "dw", "mxqtw": "qtw"}


def solve_record(arith, A, b, tol):
    t = time.time()
    if arith in MIXED:
        x, info = O.cg_solve(MIXED[arith], A, b, tol=tol, mixed=True)
    else:
        x, info = O.cg_solve(arith, A, b, tol=tol)
    nb = float(np.linalg.norm(b))
    va = "fp64" if arith in MIXED else arith
    return {"status": info["status"], "iters": int(info["iters"]), "rel_res": float(info["rel_res"]),
            "true_rel_res": O.true_residual(va, A, b, x) / nb, "oracle_seconds": round(time.time() - t, 1)}


def c4_sample(B):
    """Indices of the four largest systems and four of median size."""
    sizes = np.diff(B.sys_row_off)
    order = np.argsort(sizes, kind="stable")
    mid = len(order) // 2
    return [int(s) for s in list(order[-4:]) + list(order[mid - 2:mid + 2])]


def main(which):
    if "c2" in which:
        A, b, _ = P.case_poisson3d(128)
        path = os.path.join(HERE, "c2_oracle_solves.json")
        out = {"workload": "3D 7-point Poisson 128^3, x* ~ U[-1,1] seed 2, b = A x*, x0 = 0, tol 1e-12",
               "n": A.n, "nnz": A.nnz, "oracle_threads": O.num_threads(), "solves": {}}
        if os.path.exists(path):  # keep the solves already stored (deterministic)
            out["solves"] = json.load(open(path))["solves"]
        for ar in ("fp64", "dw", "qdw", "tw", "qtw", "qw", "qqw", "qtwe", "mxdw", "mxqtw"):
            if ar in out["solves"]:
                continue
            out["solves"][ar] = solve_record(ar, A, b, 1e-12)
            print(ar, out["solves"][ar], flush=True)
            json.dump(out, open(path, "w"), indent=1)
    if "c4" in which:
        B = P.batch_systems()
        sample = c4_sample(B)
        out = {"workload": "512-system batch (seed 4), tol 1e-12, x0 = 0; the four largest systems and four "
                           "of median size", "systems": {}}
        for s in sample:
            A, b = B.system(s)
            rec = {"n": A.n, "nnz": A.nnz, "kind": B.kinds[s]}
            for ar in ("dw", "qtw"):
                rec[ar] = solve_record(ar, A, b, 1e-12)
            out["systems"][str(s)] = rec
            print(s, rec, flush=True)
        json.dump(out, open(os.path.join(HERE, "c4_oracle_solves.json"), "w"), indent=1)
    if "c5" in which:
        Q = P.adjoint_problem(nx=100)
        A = Q.matrix()
        t = time.time()
        xo, io = O.cg_solve("qtw", A, Q.b, tol=1e-26)
        g = O.elementwise("qtw", "tofp64", xo) - Q.x_target
        lo, il = O.cg_solve("qtw", A, g, tol=1e-26)
        gt = -O.elementwise("qtw", "tofp64", O.elementwise("qtw", "mul", lo, xo))
        gb = O.elementwise("qtw", "tofp64", lo)
        rng = np.random.default_rng(5555)
        ith = rng.choice(A.n, 64, replace=False)
        ib = rng.choice(A.n, 64, replace=False)
        out = {"workload": "3D Laplacian 100^3 + diag(theta) (seeds 5, 555, 55), loss 0.5 ||x - x_target||^2, "
                           "QTW solves to 1e-26",
               "forward": {"status": io["status"], "iters": int(io["iters"])},
               "adjoint": {"status": il["status"], "iters": int(il["iters"])},
               "theta_index": [int(i) for i in ith], "theta_grad": [float(gt[i]) for i in ith],
               "b_index": [int(i) for i in ib], "b_grad": [float(gb[i]) for i in ib],
               "theta_grad_absmax": float(np.abs(gt).max()), "b_grad_absmax": float(np.abs(gb).max()),
               "oracle_seconds": round(time.time() - t, 1)}
        print({k: out[k] for k in ("forward", "adjoint", "oracle_seconds")}, flush=True)
        json.dump(out, open(os.path.join(HERE, "c5_oracle_gradient.json"), "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c4"])
