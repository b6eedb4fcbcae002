"""The C ABI from plain C: tests/capi/cg_from_c.c includes only mw.h and the
HIP runtime's C API, allocates device memory itself and calls mw_spmv,
mw_axpy, mw_dot and mw_cg_solve (no PyTorch).  Without a GPU it is compiled
and linked against libmwcg.so with gcc (the header is valid C); on the GPU
it runs and checks exact SpMV / AXPY / dot results, a QTW CG solve and two
argument errors itself."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "capi", "cg_from_c.c")
LIBDIR = os.path.join(ROOT, "paper_2510_13536_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(out):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    if not os.path.exists(os.path.join(LIBDIR, "libmwcg.so")):
        pytest.fail("libmwcg.so is not built")
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), SRC,
           "-L" + LIBDIR, "-lmwcg", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath," + LIBDIR, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return out


def test_c_caller_compiles_and_links(tmp_path):
    _build(str(tmp_path / "cg_from_c"))


@pytest.mark.gpu
def test_c_caller_runs(tmp_path):
    exe = _build(str(tmp_path / "cg_from_c"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("capi ok: QTW CG"), r.stdout
