"""The C-ABI library loads and exports every entry point include/mw.h
declares; argument validation and sizing run without a GPU (no compute)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mw.h")
LIB = os.path.join(ROOT, "paper_2510_13536_amd", "libmwcg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mw_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmwcg.so is not built (python -m paper_2510_13536_amd.build)")
    return C.CDLL(LIB)


def test_header_declares_the_core_calls():
    names = declared_functions()
    for f in ("mw_spmv", "mw_dot", "mw_axpy", "mw_cg_solve", "mw_words", "mw_elementwise"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_words_and_status_strings(lib):
    assert [lib.mw_words(a) for a in range(10)] == [1, 2, 2, 3, 3, 3, 4, 4, 1, 1]
    assert [lib.mw_scalar_words(a) for a in range(10)] == [1, 2, 2, 3, 3, 3, 4, 4, 2, 3]
    assert lib.mw_words(10) == -1 and lib.mw_scalar_words(10) == -1
    lib.mw_status_string.restype = C.c_char_p
    assert lib.mw_status_string(0) == b"ok"
    assert b"invalid" in lib.mw_status_string(-1)


def test_workspace_sizes(lib):
    lib.mw_cg_workspace_bytes.restype = C.c_size_t
    lib.mw_dot_workspace_bytes.restype = C.c_size_t
    n = 4096
    for a, k in enumerate([1, 2, 2, 3, 3]):
        ws = lib.mw_cg_workspace_bytes(a, n, 20224)
        assert ws >= 3 * k * n * 8 and ws % 256 == 0
        assert lib.mw_dot_workspace_bytes(a, n) >= 8 * k
    assert lib.mw_cg_workspace_bytes(99, n, 0) == 0
    assert lib.mw_cg_workspace_bytes(0, 0, 0) == 0


MW_MAX_N = 2 ** 31 - 2 ** 16  # include/mw.h


def test_max_n_matches_the_header():
    text = open(HEADER).read()
    assert int(re.search(r"#define MW_MAX_N (\d+)", text).group(1)) == MW_MAX_N


def test_sizes_at_the_limit(lib):
    """n = nnz = MW_MAX_N (2^31 - 2^16): every byte count is formed in 64
    bits (an FP64 workspace is then ~128 GB and a QTW one ~283 GB, with the
    SpMV plan's 59 GB), the plan and shape helpers stay consistent; one more
    is rejected."""
    lib.mw_cg_workspace_bytes.restype = C.c_size_t
    lib.mw_spmv_plan_bytes.restype = C.c_size_t
    lib.mw_cg_batched_workspace_bytes.restype = C.c_size_t
    lib.mw_dot_workspace_bytes.restype = C.c_size_t
    big = MW_MAX_N
    for f in (lambda n, z: lib.mw_cg_workspace_bytes(4, n, z), lambda n, z: lib.mw_spmv_plan_bytes(n, z),
              lambda n, z: lib.mw_cg_batched_workspace_bytes(4, 1, n, z)):
        assert f(big, big) > 0 and f(big + 1, big) == 0 and f(big, big + 1) == 0
    assert lib.mw_dot_workspace_bytes(4, big) > 0 and lib.mw_dot_workspace_bytes(4, big + 1) == 0
    for a, k in enumerate([1, 2, 2, 3, 3, 3]):
        ws = lib.mw_cg_workspace_bytes(a, big, big)
        assert ws >= 3 * k * big * 8 and ws % 256 == 0
        assert ws > lib.mw_cg_workspace_bytes(a, big // 2, big // 2)
        assert lib.mw_cg_batched_workspace_bytes(a, 1, big, big) >= 3 * k * big * 8
    for a, base in ((8, 1), (9, 4)):  # mixed types: FP64 vector planes, multi-word scalars
        wb = lib.mw_cg_batched_workspace_bytes(a, 1, big, big)
        assert 3 * big * 8 <= wb < lib.mw_cg_batched_workspace_bytes(base, 1, big, big)
    assert lib.mw_spmv_plan_bytes(big, big) >= 12 * big
    class Shape(C.Structure):
        _fields_ = [("spmv_grid", C.c_int32), ("update_grid", C.c_int32), ("update_threads", C.c_int32),
                    ("chunk", C.c_int32), ("lanes", C.c_int32), ("us_per_iteration", C.c_double)]
    lib.mw_cg_shape.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Shape)]
    sh = Shape()
    assert lib.mw_cg_shape(4, big, big, 0, C.byref(sh)) == 0
    assert (sh.spmv_grid, sh.update_grid, sh.lanes) == (1536, 1024, 0)
    assert lib.mw_cg_shape(4, big + 1, big, 0, C.byref(sh)) == -1
    vp = C.c_void_p
    lib.mw_elementwise.argtypes = [C.c_int, C.c_int, C.c_int32, vp, vp, vp, vp]
    lib.mw_axpy.argtypes = [C.c_int, C.c_int32, vp, vp, vp, vp]
    lib.mw_dot.argtypes = [C.c_int, C.c_int32, vp, vp, vp, vp, vp]
    lib.mw_csr_check.argtypes = [vp, vp]
    bogus = vp(0x1000)
    assert lib.mw_elementwise(4, 0, big + 1, bogus, bogus, bogus, None) == -1
    assert lib.mw_axpy(4, big + 1, bogus, bogus, bogus, None) == -1
    assert lib.mw_dot(4, big + 1, bogus, bogus, bogus, bogus, None) == -1

    class Csr(C.Structure):
        _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", vp), ("col_idx", vp), ("val", vp)]
    lib.mw_last_error.restype = C.c_char_p
    for n, nnz in ((big + 1, 10), (10, big + 1)):
        assert lib.mw_csr_check(C.byref(Csr(n, nnz, bogus, bogus, bogus)), None) == -1
        assert b"MW_MAX_N" in lib.mw_last_error()


def test_invalid_arguments_rejected_without_gpu(lib):
    vp = C.c_void_p
    lib.mw_elementwise.argtypes = [C.c_int, C.c_int, C.c_int32, vp, vp, vp, vp]
    lib.mw_axpy.argtypes = [C.c_int, C.c_int32, vp, vp, vp, vp]
    lib.mw_dot.argtypes = [C.c_int, C.c_int32, vp, vp, vp, vp, vp]
    lib.mw_spmv.argtypes = [C.c_int, vp, vp, vp, vp]
    lib.mw_cg_solve.argtypes = [C.c_int, vp, vp, vp, C.c_double, C.c_int32, vp, vp, vp, vp]
    bogus = vp(0x1000)
    assert lib.mw_elementwise(99, 0, 10, bogus, bogus, bogus, None) == -1  # arith
    assert lib.mw_elementwise(8, 0, 10, bogus, bogus, bogus, None) == -1   # mixed: no element-wise ops
    assert lib.mw_elementwise(1, 9, 10, bogus, bogus, bogus, None) == -1   # op
    assert lib.mw_elementwise(1, 0, -1, bogus, bogus, bogus, None) == -1   # n
    assert lib.mw_elementwise(1, 0, 10, bogus, None, bogus, None) == -1    # v needed
    assert lib.mw_elementwise(1, 0, 0, None, None, None, None) == 0        # empty: no-op
    assert lib.mw_axpy(1, 10, None, bogus, bogus, None) == -1
    assert lib.mw_dot(1, 10, bogus, bogus, bogus, None, None) == -1        # workspace
    assert lib.mw_spmv(1, None, bogus, bogus, None) == -1
    assert lib.mw_cg_solve(1, None, bogus, bogus, 1e-12, 10, None, bogus, None, None) == -1


def test_dot_noalloc_rejections_without_gpu(lib):
    """The allocation-free dot checks its arguments and its size limit on
    the host, before any device call."""
    vp = C.c_void_p
    lib.mw_dot_noalloc.argtypes = [C.c_int, C.c_int32, vp, vp, vp, vp]
    lib.mw_last_error.restype = C.c_char_p
    bogus = vp(0x1000)
    assert lib.mw_dot_noalloc(99, 10, bogus, bogus, bogus, None) == -1         # arith
    assert lib.mw_dot_noalloc(4, -1, bogus, bogus, bogus, None) == -1         # n
    assert lib.mw_dot_noalloc(4, 10, bogus, bogus, None, None) == -1          # result
    assert lib.mw_dot_noalloc(4, 10, None, bogus, bogus, None) == -1          # x
    assert lib.mw_dot_noalloc(4, 33554433, bogus, bogus, bogus, None) == -1   # beyond the scratch array
    assert b"MW_DOT_NOALLOC_MAX_N" in lib.mw_last_error()


class Shape(C.Structure):
    _fields_ = [("spmv_grid", C.c_int32), ("update_grid", C.c_int32), ("update_threads", C.c_int32),
                ("chunk", C.c_int32), ("lanes", C.c_int32), ("us_per_iteration", C.c_double)]


def test_builtin_launch_shapes(lib):
    # host-side shape resolution: no tuned entry, no GPU work
    for v in ("MW_SGRID", "MW_UGRID", "MW_UNT"):
        assert v not in os.environ
    lib.mw_cg_shape.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Shape)]
    sh = Shape()
    n, nnz = 128 ** 3, 14581760
    for a in range(6):
        assert lib.mw_cg_shape(a, n, nnz, 0, C.byref(sh)) == 0
        assert sh.spmv_grid == (1536 if a == 4 else 2048)
        assert (sh.update_grid, sh.update_threads, sh.chunk, sh.lanes, sh.us_per_iteration) == (1024, 256, 32, 0, 0.0)
    # a small matrix clamps the grids to its tiles: 4096 rows = 16 tiles of 4 slices, 16 update blocks
    assert lib.mw_cg_shape(4, 4096, 20224, 0, C.byref(sh)) == 0
    assert (sh.spmv_grid, sh.update_grid) == (16, 16)
    assert lib.mw_cg_shape(4, 4096, 20224, 3, C.byref(sh)) == 0          # batched: untuned
    assert (sh.spmv_grid, sh.chunk) == (0, 16)
    # few, long rows (18000 rows of ~381): vector rows, about 8 entries per
    # lane in FP64 (64 lanes, 4 rows per tile) and 16 otherwise (32 lanes, 8)
    for a, lanes, grid in ((0, 64, 2048), (1, 32, 2048), (4, 32, 1536)):
        assert lib.mw_cg_shape(a, 18000, 6857328, 0, C.byref(sh)) == 0
        assert (sh.lanes, sh.spmv_grid) == (lanes, grid)
    assert lib.mw_cg_shape(4, 2000, 80000, 0, C.byref(sh)) == 0      # 40 per row: 4 lanes, 64 rows per tile
    assert (sh.lanes, sh.spmv_grid) == (4, 32)
    assert lib.mw_cg_shape(4, 1 << 19, 64 << 19, 0, C.byref(sh)) == 0  # more rows: SELL-64
    assert sh.lanes == 0
    assert lib.mw_cg_shape(99, 4096, 20224, 0, C.byref(sh)) == -1
    assert lib.mw_cg_shape(4, 0, 20224, 0, C.byref(sh)) == -1


def test_invalid_shapes_and_tuner_arguments_rejected_without_gpu(lib):
    vp = C.c_void_p

    class Csr(C.Structure):
        _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", vp), ("col_idx", vp), ("val", vp)]

    class Opts(C.Structure):
        _fields_ = [("normalize", C.c_int32), ("chunk", C.c_int32), ("history", vp), ("prof", vp),
                    ("plan", vp), ("no_graph", C.c_int32), ("precond", C.c_int32), ("shape", C.POINTER(Shape))]

    bogus = vp(0x1000)
    A = Csr(64, 64, bogus, bogus, bogus)
    lib.mw_cg_solve.argtypes = [C.c_int, C.POINTER(Csr), vp, vp, C.c_double, C.c_int32, C.POINTER(Opts), vp, vp, vp]
    for bad in (Shape(4, 0, 0, 0, 0, 0.0), Shape(0, 4096, 0, 0, 0, 0.0), Shape(0, 0, 300, 0, 0, 0.0),
                Shape(0, 0, 0, 5000, 0, 0.0), Shape(0, 0, 0, 0, 3, 0.0), Shape(0, 0, 0, 0, 128, 0.0),
                Shape(0, 0, 0, 0, 1, 0.0)):
        o = Opts(1, 0, None, None, None, 0, 0, C.pointer(bad))
        assert lib.mw_cg_solve(4, C.byref(A), bogus, bogus, 1e-12, 10, C.byref(o), bogus, None, None) == -1
    for bad_pc in (2, -1):   # preconditioners: 0 (none) and 1 (Jacobi) only
        o = Opts(1, 0, None, None, None, 0, bad_pc, None)
        assert lib.mw_cg_solve(4, C.byref(A), bogus, bogus, 1e-12, 10, C.byref(o), bogus, None, None) == -1
    lib.mw_cg_tune.argtypes = [C.c_int, C.POINTER(Csr), vp, vp, C.c_int32, vp, C.POINTER(Shape), vp]
    best = Shape()
    assert lib.mw_cg_tune(4, C.byref(A), bogus, bogus, 1, bogus, C.byref(best), None) == -1      # iters
    assert lib.mw_cg_tune(4, C.byref(A), bogus, bogus, 5000, bogus, C.byref(best), None) == -1
    assert lib.mw_cg_tune(4, C.byref(A), bogus, bogus, 16, bogus, None, None) == -1             # best
    lib.mw_cg_batched_tune.argtypes = [C.c_int, C.c_int32, vp, C.POINTER(Csr), vp, vp, C.c_int32, vp,
                                       C.POINTER(Shape), vp]
    assert lib.mw_cg_batched_tune(4, 1, None, C.byref(A), bogus, bogus, 1, bogus, C.byref(best), None) == -1


def test_vector_row_plan_is_host_only_and_validates_lanes(lib):
    """mw_spmv_plan_rows fills the plan on the host (no GPU needed): lanes
    2..64 powers of two, 0 = about eight entries per lane for the average
    row; anything else is rejected."""
    vp = C.c_void_p

    class Csr(C.Structure):
        _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", vp), ("col_idx", vp), ("val", vp)]

    class Plan(C.Structure):
        _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("format", C.c_int32), ("nslices", C.c_int32),
                    ("stored", C.c_int64), ("slice_ptr", vp), ("col", vp), ("val", vp), ("slot_off", vp),
                    ("slot_mask", vp), ("ndiag", C.c_int32), ("lanes", C.c_int32), ("csr", Csr)]

    lib.mw_spmv_plan_rows.argtypes = [C.POINTER(Csr), C.c_int32, C.POINTER(Plan)]
    bogus = vp(0x1000)
    pl = Plan()
    for n, nnz, want in ((18000, 6897316, 64), (36417, 4344765, 16), (1000, 7000, 2), (1000, 40000, 8)):
        A = Csr(n, nnz, bogus, bogus, bogus)
        assert lib.mw_spmv_plan_rows(C.byref(A), 0, C.byref(pl)) == 0
        assert (pl.format, pl.lanes, pl.n, pl.nnz, pl.nslices) == (2, want, n, nnz, (n + 63) // 64)
    A = Csr(1000, 7000, bogus, bogus, bogus)
    for L in (1, 3, 128, -2):
        assert lib.mw_spmv_plan_rows(C.byref(A), L, C.byref(pl)) == -1
    assert lib.mw_spmv_plan_rows(C.byref(A), 32, C.byref(pl)) == 0 and pl.lanes == 32
    # the solver's own plan, chosen by size alone: host-only vector rows
    lib.mw_cg_plan.argtypes = [C.c_int, C.POINTER(Csr), C.c_int32, vp, C.c_size_t, C.POINTER(Plan), vp]
    A = Csr(18000, 6857328, bogus, bogus, bogus)
    for a, lanes, want in ((0, 0, 64), (4, 0, 32), (1, 0, 32), (4, 16, 16)):
        assert lib.mw_cg_plan(a, C.byref(A), lanes, None, 0, C.byref(pl), None) == 0
        assert (pl.format, pl.lanes) == (2, want)
    assert lib.mw_cg_plan(4, C.byref(A), 3, None, 0, C.byref(pl), None) == -1
    assert lib.mw_cg_plan(99, C.byref(A), 0, None, 0, C.byref(pl), None) == -1
    # plans a caller fills in are checked against their format before any GPU work
    lib.mw_spmv_planned.argtypes = [C.c_int, C.POINTER(Plan), vp, vp, vp]

    class Opts(C.Structure):
        _fields_ = [("normalize", C.c_int32), ("chunk", C.c_int32), ("history", vp), ("prof", vp),
                    ("plan", C.POINTER(Plan)), ("no_graph", C.c_int32), ("precond", C.c_int32), ("shape", vp)]

    lib.mw_cg_solve.argtypes = [C.c_int, C.POINTER(Csr), vp, vp, C.c_double, C.c_int32, C.POINTER(Opts), vp, vp, vp]
    assert lib.mw_cg_plan(4, C.byref(A), 0, None, 0, C.byref(pl), None) == 0
    for field, bad in (("lanes", 0), ("lanes", 3), ("lanes", 128), ("format", 7), ("n", 17999)):
        p2 = Plan.from_buffer_copy(pl)
        setattr(p2, field, bad)
        assert lib.mw_spmv_planned(4, C.byref(p2), bogus, vp(0x2000), None) == -1, (field, bad)
        o = Opts(1, 0, None, None, C.pointer(p2), 0, 0, None)
        assert lib.mw_cg_solve(4, C.byref(A), bogus, bogus, 1e-12, 10, C.byref(o), bogus, None, None) == -1
    p2 = Plan.from_buffer_copy(pl)
    p2.format = 1                                   # SELL64 without its arrays
    assert lib.mw_spmv_planned(4, C.byref(p2), bogus, vp(0x2000), None) == -1
