"""Host logic of bench.py, without a GPU: the one-GPU contract, the SpMV's
algorithmic byte count, and the gate that reports stored HBM traffic only
for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_spmv_bytes_is_the_csr_definition():
    # 3D Poisson 128^3: n = 2^21 rows; 7 entries per interior row, fewer on the faces
    n = 128 ** 3
    nnz = 7 * n - 6 * 128 ** 2
    assert nnz == 14581760
    assert bench.spmv_bytes(n, nnz, 3) == 12 * nnz + 4 * (n + 1) + 48 * n == 284033028
    assert bench.spmv_bytes(n, nnz, 1) - bench.spmv_bytes(n, nnz, 0) == 16 * n


def test_stored_traffic_only_for_the_profiled_sources(monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "cg_qtw_poisson3d_128_traffic.json")))
    kernel = next(iter(rec["kernels"]))
    if rec.get("source_hash") != bench.kernel_source_hash():
        pytest.skip("the committed counters were taken on other kernel sources")
    assert bench.stored_traffic(kernel) == round(rec["kernels"][kernel]["traffic_bytes"])
    assert bench.stored_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.stored_traffic(kernel) is None
