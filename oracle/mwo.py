"""ctypes binding of the CPU oracle (oracle/mwo.c) over numpy arrays.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Multi-word vectors are numpy arrays of shape (k, n), float64, C-contiguous:
plane 0 is the leading word.  A CSR matrix is any object with attributes
``n``, ``row_ptr`` (int32, n+1), ``col_idx`` (int32) and ``val`` (float64).
"""
import ctypes as C
import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

ARITH = {"fp64": 0, "dw": 1, "qdw": 2, "tw": 3, "qtw": 4, "qtwe": 5, "qw": 6, "qqw": 7}
WORDS = {"fp64": 1, "dw": 2, "qdw": 2, "tw": 3, "qtw": 3, "qtwe": 3, "qw": 4, "qqw": 4}
OPS = {"add": 0, "mul": 1, "dxmul": 2, "div": 3, "norm": 4, "neg": 5, "tofp64": 6}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -1: "einval"}

KL = 36      # limbs of the exact accumulator
KLSB = 1152  # its least significant bit weighs 2**-KLSB

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)


class CGInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32),
                ("rel_res", C.c_double), ("seconds", C.c_double)]


def _load(name):
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        from .build import build
        build()
    lib = C.CDLL(path)
    lib.mwo_words.argtypes = [C.c_int]
    lib.mwo_set_num_threads.argtypes = [C.c_int]
    lib.mwo_set_num_threads.restype = None
    lib.mwo_ops_get.restype = C.c_longlong
    lib.mwo_eft.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp, _dp]
    lib.mwo_elementwise.argtypes = [C.c_int, C.c_int, C.c_long, _dp, _dp, _dp]
    lib.mwo_spmv.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp]
    lib.mwo_dot.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp]
    lib.mwo_axpy.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp]
    lib.mwo_cg_solve.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_double,
                                 C.c_int32, C.c_int32, C.POINTER(CGInfo), _dp]
    lib.mwo_pcg_jacobi_solve.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_double,
                                         C.c_int32, C.c_int32, C.POINTER(CGInfo), _dp]
    lib.mwo_cg_solve_np.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_double,
                                    C.c_int32, C.c_int32, C.c_int32, C.POINTER(CGInfo), _dp]
    lib.mwo_cg_mixed_solve.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_double,
                                       C.c_int32, C.POINTER(CGInfo), _dp]
    lib.mwo_pcg_jacobi_mixed_solve.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_double,
                                               C.c_int32, C.POINTER(CGInfo), _dp]
    lib.mwo_exact_dot_limbs.argtypes = [C.c_int, C.c_long, _dp, _dp, _u64p]
    lib.mwo_exact_sum_limbs.argtypes = [C.c_long, _dp, _u64p]
    lib.mwo_dot_error.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp, _dp, _dp]
    lib.mwo_spmv_error.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, C.c_long,
                                   _i64p, _dp, _dp]
    lib.mwo_true_residual.argtypes = [C.c_int, C.c_long, _ip, _ip, _dp, _dp, _dp, _dp]
    return lib


_lib = None
_lib_count = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load("libmwo.so")
    return _lib


def lib_count():
    global _lib_count
    if _lib_count is None:
        _lib_count = _load("libmwo_count.so")
    return _lib_count


def num_threads():
    return lib().mwo_num_threads()


def set_num_threads(n):
    """Threads of the oracle's parallel loops (timing only; results do not
    depend on it)."""
    lib().mwo_set_num_threads(int(n))


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _planes(x, k, n=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x.reshape(1, -1)
    if x.shape[0] < k:
        x = np.concatenate([x, np.zeros((k - x.shape[0], x.shape[1]))], axis=0)
    x = np.ascontiguousarray(x[:k])
    if n is not None and x.shape[1] != n:
        raise ValueError("length mismatch")
    return x


def _csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    return int(A.n), rp, ci, va


def _check(rc):
    if rc < 0:
        raise ValueError("oracle rejected the arguments (%d)" % rc)
    return rc


# ---------------------------------------------------------------- primitives

def eft(which, a, b):
    """which: 'two_sum' | 'quick_two_sum' | 'two_prod'. Returns (x, y)."""
    w = {"two_sum": 0, "quick_two_sum": 1, "two_prod": 2}[which]
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(a)
    y = np.empty_like(a)
    _check(lib().mwo_eft(w, a.size, _d(a), _d(b), _d(x), _d(y)))
    return x, y


def elementwise(arith, op, u, v=None, count_ops=False):
    """Element-wise op over word planes; returns (k, n) (or (n,) for tofp64).

    With count_ops=True runs the op-counting build and returns
    (result, number of FP64 operations)."""
    k = WORDS[arith]
    opc = OPS[op]
    if op == "dxmul":
        uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
    else:
        uu = _planes(u, k)
    n = uu.shape[-1]
    vv = _planes(v, k, n) if v is not None else np.zeros((k, n))
    out = np.zeros(n) if op == "tofp64" else np.zeros((k, n))
    L = lib_count() if count_ops else lib()
    if count_ops:
        L.mwo_ops_reset()
    _check(L.mwo_elementwise(ARITH[arith], opc, n, _d(uu), _d(vv), _d(out)))
    if count_ops:
        return out, L.mwo_ops_get()
    return out


def spmv(arith, A, x):
    k = WORDS[arith]
    n, rp, ci, va = _csr(A)
    xx = _planes(x, k, n)
    y = np.zeros((k, n))
    _check(lib().mwo_spmv(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(xx), _d(y)))
    return y


def dot(arith, x, y):
    k = WORDS[arith]
    xx = _planes(x, k)
    yy = _planes(y, k, xx.shape[1])
    r = np.zeros(k)
    _check(lib().mwo_dot(ARITH[arith], xx.shape[1], _d(xx), _d(yy), _d(r)))
    return r


def axpy(arith, alpha, x, y):
    """Returns y + alpha * x (alpha: k words)."""
    k = WORDS[arith]
    xx = _planes(x, k)
    yy = _planes(y, k, xx.shape[1]).copy()
    al = np.zeros(k)
    a = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    al[:min(k, a.size)] = a[:k]
    _check(lib().mwo_axpy(ARITH[arith], xx.shape[1], _d(al), _d(xx), _d(yy)))
    return yy


def cg_solve(arith, A, b, x0=None, tol=1e-12, maxit=None, normalise=True, history=False, precond=None,
             mixed=False, normalise_p=False):
    """CG per the oracle.  Returns (x (k, n), info dict).

    mixed=True (an arithmetic of two or more words): FP64 vectors, the SpMV
    rows and the dots accumulated in the arithmetic (mwo_cg_mixed_solve;
    with precond="jacobi", mwo_pcg_jacobi_mixed_solve, z_i = fl(d_i r_i));
    x is then one FP64 plane (1, n); normalise does not apply.

    normalise (QDW/QTW): True / 1 normalises r every iteration (Sec. IV-D),
    False / 0 never; an integer K > 1 in iterations K, 2K, ...
    precond: None (Alg. 1) or "jacobi" (preconditioned CG with the FP64
    reciprocal diagonal, mwo_pcg_jacobi_solve).
    normalise_p (plain CG): also normalise p in the iterations that
    normalise r (a placement variant, not the paper's)."""
    if precond not in (None, "jacobi"):
        raise ValueError("precond must be None or 'jacobi'")
    if mixed and (WORDS[arith] < 2 or normalise_p):
        raise ValueError("mixed needs a multi-word arithmetic (and has no p normalisation)")
    k = 1 if mixed else WORDS[arith]
    n, rp, ci, va = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    if b.size != n:
        raise ValueError("b length mismatch")
    x = np.zeros((k, n)) if x0 is None else _planes(x0, k, n).copy()
    if maxit is None:
        maxit = 10 * n
    info = CGInfo()
    hist = np.zeros(max(int(maxit), 1)) if history else None
    if mixed:
        fn = lib().mwo_pcg_jacobi_mixed_solve if precond == "jacobi" else lib().mwo_cg_mixed_solve
        rc = fn(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(b), _d(x), float(tol),
                int(maxit), C.byref(info), _d(hist) if history else None)
    elif normalise_p:
        if precond is not None:
            raise ValueError("normalise_p applies to plain CG")
        rc = lib().mwo_cg_solve_np(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(b), _d(x), float(tol),
                                   int(maxit), int(normalise), 1, C.byref(info), _d(hist) if history else None)
    else:
        fn = lib().mwo_pcg_jacobi_solve if precond == "jacobi" else lib().mwo_cg_solve
        rc = fn(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(b), _d(x), float(tol),
                int(maxit), int(normalise), C.byref(info), _d(hist) if history else None)
    _check(rc)
    out = {"iters": info.iters, "status": STATUS[info.status], "status_code": info.status,
           "rel_res": info.rel_res}
    if history:
        out["history"] = hist[:info.iters].copy()
    return x, out


# ---------------------------------------------------------- exact references

def _limbs_to_fraction(limbs):
    v = 0
    for i in range(KL - 1, -1, -1):
        v = (v << 64) | int(limbs[i])
    if v >> (64 * KL - 1):
        v -= 1 << (64 * KL)
    return Fraction(v, 1 << KLSB)


def exact_sum(t):
    """Exact sum of float64 values, as a Fraction (long accumulator)."""
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
    limbs = np.zeros(KL, dtype=np.uint64)
    _check(lib().mwo_exact_sum_limbs(t.size, _d(t), limbs.ctypes.data_as(_u64p)))
    return _limbs_to_fraction(limbs)


def exact_dot(arith, x, y):
    """Exact x^T y of k-word vectors (all word products), as a Fraction."""
    k = WORDS[arith]
    xx = _planes(x, k)
    yy = _planes(y, k, xx.shape[1])
    limbs = np.zeros(KL, dtype=np.uint64)
    _check(lib().mwo_exact_dot_limbs(ARITH[arith], xx.shape[1], _d(xx), _d(yy),
                                     limbs.ctypes.data_as(_u64p)))
    return _limbs_to_fraction(limbs)


def dot_error(arith, x, y, res):
    """(|res - x^T y|, sum_i |x_i y_i|) with the difference formed exactly."""
    k = WORDS[arith]
    xx = _planes(x, k)
    yy = _planes(y, k, xx.shape[1])
    rr = np.zeros(k)
    r = np.atleast_1d(np.asarray(res, dtype=np.float64))
    rr[:min(k, r.size)] = r[:k]
    e = C.c_double()
    s = C.c_double()
    _check(lib().mwo_dot_error(ARITH[arith], xx.shape[1], _d(xx), _d(yy), _d(rr),
                               C.byref(e), C.byref(s)))
    return e.value, s.value


def spmv_error(arith, A, x, y, rows=None):
    """Per-row (|y_i - (Ax)_i|, sum_j |a_ij x_j|) for the given rows."""
    k = WORDS[arith]
    n, rp, ci, va = _csr(A)
    xx = _planes(x, k, n)
    yy = _planes(y, k, n)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    err = np.zeros(rows.size)
    sc = np.zeros(rows.size)
    _check(lib().mwo_spmv_error(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(xx), _d(yy),
                                rows.size, rows.ctypes.data_as(_i64p), _d(err), _d(sc)))
    return err, sc


def true_residual(arith, A, b, x):
    """||b - A x||_2 with every row residual formed exactly."""
    k = WORDS[arith]
    n, rp, ci, va = _csr(A)
    xx = _planes(x, k, n)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    out = C.c_double()
    _check(lib().mwo_true_residual(ARITH[arith], n, _i(rp), _i(ci), _d(va), _d(b), _d(xx),
                                   C.byref(out)))
    return out.value


def fraction_of(x):
    """Exact value of a multi-word number given as a sequence of words."""
    return sum((Fraction(float(w)) for w in np.atleast_1d(x)), Fraction(0))
