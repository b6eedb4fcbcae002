"""Thin Python binding of libmwcg (C ABI in include/mw.h).

Argument marshalling only: every arithmetic step runs in the HIP kernels of
libmwcg.so.  PyTorch provides device memory (tensors) and the stream
(torch.cuda.current_stream()).  There is no CPU fallback: if the library is
not built, or no GPU is present, the calls raise.

Multi-word vectors are float64 CUDA tensors of shape (k, n) (k word planes,
plane 0 the leading word); k-word scalars are float64 tensors of shape (k,).
"""
import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmwcg.so")

ARITH = {"fp64": 0, "dw": 1, "qdw": 2, "tw": 3, "qtw": 4, "qtwe": 5, "qw": 6, "qqw": 7, "mxdw": 8, "mxqtw": 9}
# planes of a vector element
WORDS = {"fp64": 1, "dw": 2, "qdw": 2, "tw": 3, "qtw": 3, "qtwe": 3, "qw": 4, "qqw": 4, "mxdw": 1, "mxqtw": 1}
# words of a scalar (a dot result, an axpy alpha): multi-word for the mixed types
SWORDS = dict(WORDS, mxdw=2, mxqtw=3)
DOT_NOALLOC_MAX_N = 33554432  # MW_DOT_NOALLOC_MAX_N in include/mw.h
OPS = {"add": 0, "mul": 1, "dxmul": 2, "div": 3, "norm": 4, "neg": 5, "tofp64": 6}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown"}
MW_EINVAL, MW_EHIP = -1, -2

_vp = C.c_void_p


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", _vp), ("col_idx", _vp), ("val", _vp)]


class CgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("seconds", C.c_double)]


PROF_CLASSES = ("spmv", "update_r", "update_p", "final")


class CgProf(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_int64 * 4), ("mask", C.c_int32),
                ("reserved", C.c_int32)]

    @classmethod
    def of(cls, *classes):
        """A timing request for the named classes (none named: all)."""
        p = cls()
        p.mask = sum(1 << PROF_CLASSES.index(c) for c in classes)
        return p

    def as_dict(self):
        return {c: {"ms": self.ms[i], "launches": self.launches[i],
                    "avg_us": 1e3 * self.ms[i] / self.launches[i] if self.launches[i] else None}
                for i, c in enumerate(PROF_CLASSES)}


FMT = {0: "csr", 1: "sell64", 2: "csrvec"}


class SpmvPlan(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("format", C.c_int32), ("nslices", C.c_int32),
                ("stored", C.c_int64), ("slice_ptr", _vp), ("col", _vp), ("val", _vp), ("slot_off", _vp),
                ("slot_mask", _vp), ("ndiag", C.c_int32), ("lanes", C.c_int32), ("csr", Csr)]


class Shape(C.Structure):
    """Launch shape (mw_shape_t); a field <= 0 is "not set"."""
    _fields_ = [("spmv_grid", C.c_int32), ("update_grid", C.c_int32), ("update_threads", C.c_int32),
                ("chunk", C.c_int32), ("lanes", C.c_int32), ("us_per_iteration", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    @classmethod
    def of(cls, shape):
        """A Shape from a Shape, a dict of its fields, or None."""
        if shape is None or isinstance(shape, cls):
            return shape
        return cls(**{f: shape.get(f, 0) for f, _ in cls._fields_})


class CgOpts(C.Structure):
    _fields_ = [("normalize", C.c_int32), ("chunk", C.c_int32), ("history", _vp),
                ("prof", C.POINTER(CgProf)), ("plan", C.POINTER(SpmvPlan)), ("no_graph", C.c_int32),
                ("precond", C.c_int32), ("shape", C.POINTER(Shape)), ("normalize_p", C.c_int32)]


PRECOND = {None: 0, "jacobi": 1}
MAX_N = 2 ** 31 - 2 ** 16   # MW_MAX_N: the largest n and nnz the library takes
MAXIT_MAX = 2 ** 31 - 1     # maxit is an int32


class MWError(RuntimeError):
    pass


_lib = None


def _hip_runtimes_mapped():
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def lib():
    """The loaded libmwcg (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MWError("libmwcg.so is not built (run: python -m paper_2510_13536_amd.build)")
    L = C.CDLL(LIB_PATH)
    rt = _hip_runtimes_mapped()
    if len(rt) > 1:
        raise MWError("two HIP runtimes are mapped in this process: %s" % sorted(rt))
    L.mw_words.argtypes = [C.c_int]
    L.mw_scalar_words.argtypes = [C.c_int]
    L.mw_status_string.restype = C.c_char_p
    L.mw_last_error.restype = C.c_char_p
    L.mw_elementwise.argtypes = [C.c_int, C.c_int, C.c_int32, _vp, _vp, _vp, _vp]
    L.mw_axpy.argtypes = [C.c_int, C.c_int32, _vp, _vp, _vp, _vp]
    L.mw_dot_workspace_bytes.argtypes = [C.c_int, C.c_int32]
    L.mw_dot_workspace_bytes.restype = C.c_size_t
    L.mw_dot.argtypes = [C.c_int, C.c_int32, _vp, _vp, _vp, _vp, _vp]
    L.mw_dot_noalloc.argtypes = [C.c_int, C.c_int32, _vp, _vp, _vp, _vp]
    L.mw_spmv.argtypes = [C.c_int, C.POINTER(Csr), _vp, _vp, _vp]
    L.mw_spmv_plan_bytes.argtypes = [C.c_int32, C.c_int32]
    L.mw_spmv_plan_bytes.restype = C.c_size_t
    L.mw_spmv_plan.argtypes = [C.POINTER(Csr), _vp, C.c_size_t, C.POINTER(SpmvPlan), _vp]
    L.mw_spmv_planned.argtypes = [C.c_int, C.POINTER(SpmvPlan), _vp, _vp, _vp]
    L.mw_spmv_plan_rows.argtypes = [C.POINTER(Csr), C.c_int32, C.POINTER(SpmvPlan)]
    L.mw_csr_check.argtypes = [C.POINTER(Csr), _vp]
    L.mw_cg_plan.argtypes = [C.c_int, C.POINTER(Csr), C.c_int32, _vp, C.c_size_t, C.POINTER(SpmvPlan), _vp]
    L.mw_cg_workspace_bytes.argtypes = [C.c_int, C.c_int32, C.c_int32]
    L.mw_cg_workspace_bytes.restype = C.c_size_t
    L.mw_cg_solve.argtypes = [C.c_int, C.POINTER(Csr), _vp, _vp, C.c_double, C.c_int32,
                              C.POINTER(CgOpts), _vp, C.POINTER(CgInfo), _vp]
    L.mw_csr_grad.argtypes = [C.c_int, C.POINTER(Csr), _vp, _vp, _vp, _vp]
    L.mw_cg_batched_workspace_bytes.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int32]
    L.mw_cg_batched_workspace_bytes.restype = C.c_size_t
    L.mw_cg_solve_batched.argtypes = [C.c_int, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Csr), _vp, _vp,
                                      C.c_double, C.c_int32, C.POINTER(CgOpts), _vp, _vp, _vp, _vp,
                                      C.POINTER(CgInfo), _vp]
    L.mw_cg_tune.argtypes = [C.c_int, C.POINTER(Csr), _vp, _vp, C.c_int32, _vp, C.POINTER(Shape), _vp]
    L.mw_cg_batched_tune.argtypes = [C.c_int, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Csr), _vp, _vp,
                                     C.c_int32, _vp, C.POINTER(Shape), _vp]
    L.mw_cg_shape.argtypes = [C.c_int, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Shape)]
    _lib = L
    return L


def _check(rc, what):
    if rc < 0:
        msg = lib().mw_status_string(rc).decode()
        detail = lib().mw_last_error().decode()
        if detail:
            msg += ": " + detail
        raise MWError("%s failed (%d): %s" % (what, rc, msg))
    return rc


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else None


def _vec(t, k, n=None, name="vector"):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise MWError("%s must be a float64 CUDA tensor" % name)
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() != 2 or t.shape[0] != k or (n is not None and t.shape[1] != n) or not t.is_contiguous():
        raise MWError("%s must be a contiguous (%d, n) tensor, got %s" % (name, k, tuple(t.shape)))
    return t


def words(arith):
    return WORDS[arith]


class DeviceCSR:
    """FP64 CSR matrix resident on the GPU (int32 indices)."""

    def __init__(self, n, row_ptr, col_idx, val):
        self.n = int(n)
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val
        self.nnz = int(col_idx.numel())
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32 or val.dtype != torch.float64:
            raise MWError("CSR arrays must be int32/int32/float64")
        if row_ptr.numel() != self.n + 1 or val.numel() != self.nnz:
            raise MWError("CSR array sizes are inconsistent")

    @classmethod
    def from_host(cls, A, device="cuda"):
        """From any object with n, row_ptr, col_idx, val (numpy arrays)."""
        return cls(A.n, torch.as_tensor(A.row_ptr, dtype=torch.int32, device=device).contiguous(),
                   torch.as_tensor(A.col_idx, dtype=torch.int32, device=device).contiguous(),
                   torch.as_tensor(A.val, dtype=torch.float64, device=device).contiguous())

    def c(self):
        return Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())


def elementwise(arith, op, u, v=None, out=None):
    """w = op(u, v) over word planes; op in OPS."""
    k = WORDS[arith]
    if op == "dxmul":
        u = u.reshape(1, -1)
        if not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise MWError("u must be a contiguous float64 CUDA tensor")
    else:
        u = _vec(u, k, name="u")
    n = u.shape[1]
    if v is not None:
        v = _vec(v, k, n, name="v")
    if out is None:
        out = torch.empty((1 if op == "tofp64" else k, n), dtype=torch.float64, device=u.device)
    _check(lib().mw_elementwise(ARITH[arith], OPS[op], n, _ptr(u), _ptr(v), _ptr(out), _stream()),
           "mw_elementwise")
    return out


def axpy(arith, alpha, x, y):
    """y += alpha * x in place; alpha: (SWORDS[arith],) device tensor."""
    k = WORDS[arith]
    x = _vec(x, k, name="x")
    y = _vec(y, k, x.shape[1], name="y")
    alpha = alpha.reshape(-1)
    if alpha.numel() != SWORDS[arith] or not alpha.is_cuda or alpha.dtype != torch.float64:
        raise MWError("alpha must be a (%d,) float64 CUDA tensor" % SWORDS[arith])
    _check(lib().mw_axpy(ARITH[arith], x.shape[1], _ptr(alpha.contiguous()), _ptr(x), _ptr(y), _stream()),
           "mw_axpy")
    return y


def dot(arith, x, y, out=None, workspace=None):
    """x^T y as a (SWORDS[arith],) device tensor."""
    k = WORDS[arith]
    x = _vec(x, k, name="x")
    y = _vec(y, k, x.shape[1], name="y")
    n = x.shape[1]
    if out is None:
        out = torch.empty(SWORDS[arith], dtype=torch.float64, device=x.device)
    need = lib().mw_dot_workspace_bytes(ARITH[arith], n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check(lib().mw_dot(ARITH[arith], n, _ptr(x), _ptr(y), _ptr(out), _ptr(workspace), _stream()), "mw_dot")
    return out


def dot_noalloc(arith, x, y, out):
    """x^T y into the caller's (SWORDS[arith],) device tensor `out`, with no
    workspace and no allocation (mw_dot_noalloc; n <= DOT_NOALLOC_MAX_N)."""
    k = WORDS[arith]
    x = _vec(x, k, name="x")
    y = _vec(y, k, x.shape[1], name="y")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.is_contiguous() and out.numel() == SWORDS[arith]):
        raise MWError("out must be a contiguous (%d,) float64 CUDA tensor" % SWORDS[arith])
    _check(lib().mw_dot_noalloc(ARITH[arith], x.shape[1], _ptr(x), _ptr(y), _ptr(out), _stream()),
           "mw_dot_noalloc")
    return out


def spmv(arith, A, x, y=None):
    """y = A x; A a DeviceCSR."""
    k = WORDS[arith]
    x = _vec(x, k, A.n, name="x")
    if y is None:
        y = torch.empty_like(x)
    y = _vec(y, k, A.n, name="y")
    csr = A.c()
    _check(lib().mw_spmv(ARITH[arith], C.byref(csr), _ptr(x), _ptr(y), _stream()), "mw_spmv")
    return y


def csr_check(A):
    """Check A's CSR arrays on the device (mw_csr_check); raises MWError
    naming the first failed property."""
    csr = A.c()
    _check(lib().mw_csr_check(C.byref(csr), _stream()), "mw_csr_check")


class Plan:
    """A SpMV plan of a DeviceCSR: SELL-64 (or the CSR fallback), bit-identical
    to spmv; with rows=L (0 = chosen from the average row length) the
    vector-row format (mw_spmv_plan_rows), L lanes per row; with
    solver=arith the plan cg_solve builds for itself in that arithmetic
    (mw_cg_plan; rows then overrides its lanes per row)."""

    def __init__(self, A, rows=None, solver=None):
        self.A = A
        self.c = SpmvPlan()
        self._csr = A.c()
        if solver is not None:
            # the plan cg_solve(solver, A) builds for itself (mw_cg_plan)
            nbytes = lib().mw_spmv_plan_bytes(A.n, A.nnz)
            self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=A.val.device)
            _check(lib().mw_cg_plan(ARITH[solver], C.byref(self._csr), int(rows or 0), _ptr(self.buffer), nbytes,
                                    C.byref(self.c), _stream()), "mw_cg_plan")
            if self.c.format == 2:
                self.buffer = None
            return
        if rows is not None:
            self.buffer = None
            _check(lib().mw_spmv_plan_rows(C.byref(self._csr), int(rows), C.byref(self.c)), "mw_spmv_plan_rows")
            return
        nbytes = lib().mw_spmv_plan_bytes(A.n, A.nnz)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=A.val.device)
        _check(lib().mw_spmv_plan(C.byref(self._csr), _ptr(self.buffer), nbytes, C.byref(self.c), _stream()),
               "mw_spmv_plan")

    @property
    def lanes(self):
        """Lanes per row (vector-row plans only)."""
        return int(self.c.lanes)

    @property
    def format(self):
        return FMT[self.c.format]

    @property
    def stored(self):
        return int(self.c.stored)

    @property
    def ndiag(self):
        """Slices stored as diagonal slots (SELL-64 only)."""
        return int(self.c.ndiag)


def spmv_planned(arith, plan, x, y=None):
    """y = A x with a Plan (bit-identical to spmv, except for vector-row
    plans: see Plan)."""
    k = WORDS[arith]
    x = _vec(x, k, plan.A.n, name="x")
    if y is None:
        y = torch.empty_like(x)
    y = _vec(y, k, plan.A.n, name="y")
    _check(lib().mw_spmv_planned(ARITH[arith], C.byref(plan.c), _ptr(x), _ptr(y), _stream()), "mw_spmv_planned")
    return y


def csr_grad(arith, A, lam, x, out=None):
    """grad_val[k] = -(lam_i x_j) on A's pattern (FP64, CSR order)."""
    k = WORDS[arith]
    lam = _vec(lam, k, A.n, name="lam")
    x = _vec(x, k, A.n, name="x")
    if out is None:
        out = torch.empty(A.nnz, dtype=torch.float64, device=x.device)
    csr = A.c()
    _check(lib().mw_csr_grad(ARITH[arith], C.byref(csr), _ptr(lam), _ptr(x), _ptr(out), _stream()), "mw_csr_grad")
    return out


def cg_workspace(arith, A, device=None):
    nbytes = lib().mw_cg_workspace_bytes(ARITH[arith], A.n, A.nnz)
    return torch.empty(nbytes, dtype=torch.uint8, device=device or A.val.device)


def cg_solve(arith, A, b, x=None, tol=1e-12, maxit=None, normalize=True, chunk=0, history=False,
             workspace=None, prof=None, plan=None, graph=True, shape=None, precond=None, normalize_p=False):
    """Solve A x = b by CG in `arith`.  Returns (x (k, n) tensor, info dict).

    prof: a CgProf to accumulate per-kernel device times into (optional);
    plan: a Plan of A to reuse (optional; else the solver builds its own
    per call, as Plan(A, solver=arith) does);
    graph: replay captured chunks (True) or launch kernels directly;
    shape: launch shape (Shape or dict of its fields; optional);
    precond: None (Alg. 1) or "jacobi" (preconditioned CG, M^-1 the FP64
    reciprocal diagonal);
    normalize_p: quasi types, normalise p with r (a placement variant)."""
    if precond not in PRECOND:
        raise MWError("precond must be None or 'jacobi'")
    k = WORDS[arith]
    b = b.reshape(-1)
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == A.n):
        raise MWError("b must be a contiguous float64 CUDA tensor of length n")
    if x is None:
        x = torch.zeros((k, A.n), dtype=torch.float64, device=b.device)
    x = _vec(x, k, A.n, name="x")
    if maxit is None:
        maxit = min(10 * A.n, MAXIT_MAX)
    if not 0 <= int(maxit) <= MAXIT_MAX:
        raise MWError("maxit must be in [0, 2^31 - 1]")
    if workspace is None:
        workspace = cg_workspace(arith, A, b.device)
    hist = torch.zeros(max(int(maxit), 1), dtype=torch.float64, device=b.device) if history else None
    sh = Shape.of(shape)
    opts = CgOpts(int(normalize), int(chunk), hist.data_ptr() if hist is not None else None,
                  C.pointer(prof) if prof is not None else None,
                  C.pointer(plan.c) if plan is not None else None, 0 if graph else 1, PRECOND[precond],
                  C.pointer(sh) if sh is not None else None, 1 if normalize_p else 0)
    info = CgInfo()
    csr = A.c()
    rc = lib().mw_cg_solve(ARITH[arith], C.byref(csr), _ptr(b), _ptr(x), float(tol), int(maxit),
                           C.byref(opts), _ptr(workspace), C.byref(info), _stream())
    _check(rc, "mw_cg_solve")
    out = {"iters": info.iters, "status": STATUS.get(info.status, str(info.status)),
           "status_code": info.status, "rel_res": info.rel_res, "seconds": info.seconds}
    if hist is not None:
        out["history"] = hist[:info.iters].cpu().numpy()
    return x, out


def cg_solve_batched(arith, A, sys_row_off, b, x=None, tol=1e-12, maxit=None, normalize=True, chunk=0,
                     graph=True, workspace=None, shape=None, precond=None):
    """Solve the independent systems on the diagonal blocks of A (a DeviceCSR)
    together; sys_row_off: host sequence of nsys + 1 row offsets; precond:
    None or "jacobi" (as cg_solve, per system).

    Returns (x (k, n) tensor, iters, status, rel_res (numpy arrays), info)."""
    import numpy as np
    k = WORDS[arith]
    off = np.ascontiguousarray(np.asarray(sys_row_off, dtype=np.int32))
    nsys = off.size - 1
    b = b.reshape(-1)
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == A.n):
        raise MWError("b must be a contiguous float64 CUDA tensor of length n")
    if x is None:
        x = torch.zeros((k, A.n), dtype=torch.float64, device=b.device)
    x = _vec(x, k, A.n, name="x")
    if maxit is None:
        maxit = min(10 * int(np.max(np.diff(off))), MAXIT_MAX) if nsys > 0 else 0
    if not 0 <= int(maxit) <= MAXIT_MAX:
        raise MWError("maxit must be in [0, 2^31 - 1]")
    if workspace is None:
        nbytes = lib().mw_cg_batched_workspace_bytes(ARITH[arith], nsys, A.n, A.nnz)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    iters = torch.zeros(nsys, dtype=torch.int32, device=b.device)
    status = torch.zeros(nsys, dtype=torch.int32, device=b.device)
    rel = torch.zeros(nsys, dtype=torch.float64, device=b.device)
    sh = Shape.of(shape)
    if precond not in PRECOND:
        raise MWError("precond must be None or 'jacobi'")
    opts = CgOpts(int(normalize), int(chunk), None, None, None, 0 if graph else 1, PRECOND[precond],
                  C.pointer(sh) if sh is not None else None)
    info = CgInfo()
    csr = A.c()
    rc = lib().mw_cg_solve_batched(ARITH[arith], nsys, off.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(csr),
                                   _ptr(b), _ptr(x), float(tol), int(maxit), C.byref(opts), _ptr(workspace),
                                   _ptr(iters), _ptr(status), _ptr(rel), C.byref(info), _stream())
    _check(rc, "mw_cg_solve_batched")
    return (x, iters.cpu().numpy(), status.cpu().numpy(), rel.cpu().numpy(),
            {"iters": info.iters, "status": STATUS.get(info.status, str(info.status)), "seconds": info.seconds})


def cg_tune(arith, A, b, iters=32, workspace=None):
    """Time candidate launch shapes on A (mw_cg_tune); later cg_solve calls
    on matrices of A's size use the winner.  Returns its fields (dict)."""
    b = b.reshape(-1)
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == A.n):
        raise MWError("b must be a contiguous float64 CUDA tensor of length n")
    x = torch.zeros((WORDS[arith], A.n), dtype=torch.float64, device=b.device)
    if workspace is None:
        workspace = cg_workspace(arith, A, b.device)
    best = Shape()
    csr = A.c()
    _check(lib().mw_cg_tune(ARITH[arith], C.byref(csr), _ptr(b), _ptr(x), int(iters), _ptr(workspace),
                            C.byref(best), _stream()), "mw_cg_tune")
    return best.as_dict()


def cg_batched_tune(arith, A, sys_row_off, b, iters=16, workspace=None):
    """Time candidate slice-kernel grids on a batch (mw_cg_batched_tune);
    later cg_solve_batched calls on batches of that size use the winner."""
    import numpy as np
    off = np.ascontiguousarray(np.asarray(sys_row_off, dtype=np.int32))
    nsys = off.size - 1
    b = b.reshape(-1)
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == A.n):
        raise MWError("b must be a contiguous float64 CUDA tensor of length n")
    x = torch.zeros((WORDS[arith], A.n), dtype=torch.float64, device=b.device)
    if workspace is None:
        nbytes = lib().mw_cg_batched_workspace_bytes(ARITH[arith], nsys, A.n, A.nnz)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    best = Shape()
    csr = A.c()
    _check(lib().mw_cg_batched_tune(ARITH[arith], nsys, off.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(csr),
                                    _ptr(b), _ptr(x), int(iters), _ptr(workspace), C.byref(best), _stream()),
           "mw_cg_batched_tune")
    return best.as_dict()


def cg_shape(arith, n, nnz, nsys=0):
    """(tuned, shape dict): the launch shape a solve would use now."""
    sh = Shape()
    rc = _check(lib().mw_cg_shape(ARITH[arith], int(n), int(nnz), int(nsys), C.byref(sh)), "mw_cg_shape")
    return bool(rc), sh.as_dict()
