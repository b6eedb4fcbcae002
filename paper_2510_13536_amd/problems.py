"""Seeded synthetic SPD problems in FP64 CSR form.

Input generation only: nothing here performs multi-word arithmetic.  The
same generators feed both the GPU library and the CPU oracle, and the
right-hand sides are formed once here (plain FP64 sparse matrix-vector
product) so both sides see the same bytes.

The paper evaluates CG on SuiteSparse SPD matrices with a known exact
solution (Sec. V-A, Table I).  Those matrices are not available here; the
workloads below stand in for them:
  * 2D 5-point and 3D 7-point Poisson (Dirichlet, unscaled stencil),
  * a symmetric banded random matrix made strictly diagonally dominant and
    then scaled D A D with D_ii = 10^U(-3, 3) (condition number ~1e12+),
  * weighted circulant-graph Laplacians plus a small diagonal shift,
  * a batch of uneven Poisson / circulant systems,
  * a 3D Laplacian plus a positive diagonal parameter (for gradients).
Columns are ascending inside every row and indices are int32.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """FP64 CSR matrix with int32 indices (columns ascending per row)."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    @classmethod
    def from_scipy(cls, M):
        M = sp.csr_matrix(M, dtype=np.float64)
        M.sum_duplicates()
        M.sort_indices()
        return cls(n=M.shape[0],
                   row_ptr=np.ascontiguousarray(M.indptr, dtype=np.int32),
                   col_idx=np.ascontiguousarray(M.indices, dtype=np.int32),
                   val=np.ascontiguousarray(M.data, dtype=np.float64))

    def to_scipy(self):
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def matvec(self, x):
        """FP64 product A x (input generation only)."""
        return self.to_scipy() @ np.asarray(x, dtype=np.float64)

    def bytes(self):
        return self.val.nbytes + self.col_idx.nbytes + self.row_ptr.nbytes


def _tridiag(m, diag=2.0):
    e = np.ones(m)
    return sp.diags([-e[:-1], diag * e, -e[:-1]], [-1, 0, 1], format="csr")


def poisson1d(n):
    """tridiag(-1, 2, -1) of order n."""
    return CSR.from_scipy(_tridiag(n))


def poisson2d(nx, ny=None):
    """5-point Laplacian on an nx x ny grid: diagonal 4, neighbours -1,
    natural ordering i + nx*j."""
    ny = nx if ny is None else ny
    T = _tridiag(nx, 0.0)
    S = _tridiag(ny, 0.0)
    A = sp.kron(sp.identity(ny), T) + sp.kron(S, sp.identity(nx)) + 4.0 * sp.identity(nx * ny)
    return CSR.from_scipy(A)


def poisson3d(nx, ny=None, nz=None, shift=None):
    """7-point Laplacian on an nx x ny x nz grid: diagonal 6, neighbours -1,
    ordering i + nx*(j + ny*k).  `shift` (length n) is added to the
    diagonal when given."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Tx, Ty, Tz = _tridiag(nx, 0.0), _tridiag(ny, 0.0), _tridiag(nz, 0.0)
    A = (sp.kron(Iz, sp.kron(Iy, Tx)) + sp.kron(Iz, sp.kron(Ty, Ix)) +
         sp.kron(Tz, sp.kron(Iy, Ix)))
    d = 6.0 * np.ones(nx * ny * nz)
    if shift is not None:
        d = d + np.asarray(shift, dtype=np.float64)
    A = A + sp.diags(d, 0)
    return CSR.from_scipy(A)


def banded_spd(n, half_bw=13, seed=3, dseed=33, margin=1.0, scale=True):
    """Symmetric banded random SPD matrix.

    Off-diagonals A_ij = A_ji ~ N(0, 1) on offsets 1..half_bw (drawn offset
    by offset from default_rng(seed)); A_ii = sum_{j != i} |A_ij| + margin
    (strict diagonal dominance, hence SPD).  With `scale`, returns D A D
    with D_ii = 10^U(-3, 3) drawn from default_rng(dseed)."""
    rng = np.random.default_rng(seed)
    offs, diags = [], []
    rowabs = np.zeros(n)
    for d in range(1, half_bw + 1):
        v = rng.standard_normal(n - d)
        rowabs[: n - d] += np.abs(v)
        rowabs[d:] += np.abs(v)
        offs += [d, -d]
        diags += [v, v]
    offs.append(0)
    diags.append(rowabs + margin)
    A = sp.diags(diags, offs, shape=(n, n), format="csr")
    if scale:
        D = 10.0 ** np.random.default_rng(dseed).uniform(-3.0, 3.0, n)
        Dm = sp.diags(D, 0)
        A = Dm @ A @ Dm
    return CSR.from_scipy(A)


# The paper's test matrices (Table I: SuiteSparse SPD matrices, not
# available here) by name, n and number of nonzeros.  Their stand-ins are
# banded SPD matrices (banded_spd, unscaled) of the same n and about the same
# nonzeros per row (half bandwidth (nnz/n - 1)/2): the shape that sets the
# cost of an iteration, for timing a fixed number of iterations.
TABLE1 = [("Hook_1498", 1498023, 60917445), ("bone010", 986703, 47851783), ("nd24k", 72000, 28715634),
          ("crankseg_2", 63838, 14148858), ("crankseg_1", 52804, 10614210), ("nd6k", 18000, 6897316),
          ("consph", 83334, 6010480), ("pdb1HYS", 36417, 4344765)]


def table1_standin(name, seed=70):
    """Banded SPD stand-in for the Table I matrix `name` (see TABLE1)."""
    for i, (nm, n, nnz) in enumerate(TABLE1):
        if nm == name:
            half_bw = max(1, int(round((nnz / n - 1.0) / 2.0)))
            return banded_spd(n, half_bw=half_bw, seed=seed + i, scale=False)
    raise KeyError(name)


def circulant_laplacian(n, offsets, weights, shift=1e-3):
    """Weighted circulant-graph Laplacian plus shift*I: each offset o with
    weight w links i and (i +- o) mod n.  SPD for shift > 0."""
    rows, cols, vals = [], [], []
    idx = np.arange(n)
    diag = np.full(n, shift)
    for o, w in zip(offsets, weights):
        for j in ((idx + o) % n, (idx - o) % n):
            rows.append(idx)
            cols.append(j)
            vals.append(np.full(n, -w))
        diag += 2.0 * w
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return CSR.from_scipy(A)


def uniform(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def integer_vector(n, seed, lo=-8, hi=8):
    """Integer-valued FP64 vector in [lo, hi]: with an integer stencil, b = A x
    is then exact in FP64 (a manufactured exact solution)."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.float64)


# ----------------------------------------------------------------- workloads

def case_poisson2d_64(seed=1):
    """2D 5-point Poisson 64x64 (n = 4096, nnz = 20224); x_true ~ U[-1,1]."""
    A = poisson2d(64)
    x = uniform(A.n, seed)
    return A, A.matvec(x), x


def case_poisson3d(nx=128, seed=2):
    """3D 7-point Poisson nx^3 (128^3: n = 2,097,152, nnz = 14,581,760)."""
    A = poisson3d(nx)
    x = uniform(A.n, seed)
    return A, A.matvec(x), x


def case_banded_illcond(n=1 << 20, seed=3, dseed=33, xseed=333, half_bw=13):
    """Banded ill-conditioned SPD (n = 1,048,576, 27 nnz per interior row)."""
    A = banded_spd(n, half_bw=half_bw, seed=seed, dseed=dseed)
    x = uniform(A.n, xseed)
    return A, A.matvec(x), x


@dataclass
class Batch:
    """A batch of independent systems as one block-diagonal CSR matrix.
    System s owns rows sys_row_off[s] .. sys_row_off[s+1]-1."""
    A: CSR
    sys_row_off: np.ndarray  # int32, nsys + 1
    b: np.ndarray
    x_true: np.ndarray
    kinds: list

    @property
    def nsys(self):
        return len(self.sys_row_off) - 1

    def system(self, s):
        """System s as its own CSR (local indices) plus its b."""
        r0, r1 = int(self.sys_row_off[s]), int(self.sys_row_off[s + 1])
        rp = self.A.row_ptr[r0:r1 + 1].astype(np.int64)
        z0, z1 = int(rp[0]), int(rp[-1])
        sub = CSR(n=r1 - r0, row_ptr=(rp - z0).astype(np.int32),
                  col_idx=(self.A.col_idx[z0:z1] - r0).astype(np.int32),
                  val=self.A.val[z0:z1].copy())
        return sub, self.b[r0:r1].copy()


def batch_from_systems(mats, bs, kinds=None):
    """A Batch from a list of CSR systems and their right-hand sides."""
    A = CSR.from_scipy(sp.block_diag([m.to_scipy() for m in mats], format="csr"))
    off = np.zeros(len(mats) + 1, dtype=np.int64)
    off[1:] = np.cumsum([m.n for m in mats])
    b = np.concatenate([np.asarray(v, dtype=np.float64) for v in bs])
    return Batch(A=A, sys_row_off=off.astype(np.int32), b=b, x_true=np.full(A.n, np.nan),
                 kinds=kinds or ["given"] * len(mats))


def batch_systems(nsys=512, seed=4, nmin=1024, nmax=65536):
    """Uneven batch: n_s = round(exp(U(ln nmin, ln nmax))).  Even s: Poisson,
    2D for s % 4 == 0 (nx = round(sqrt n), ny = round(n / nx)), 3D for
    s % 4 == 2 (nx = ny = round(cbrt n), nz = round(n / nx^2)).  Odd s:
    circulant-graph Laplacian + 1e-3 I with m ~ U{4..13} distinct offsets in
    [1, n/2) and weights U(0.1, 1].  x_true_s ~ U[-1, 1] (seed 4000 + s)."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), nsys))).astype(int)
    mats, kinds = [], []
    for s in range(nsys):
        n = int(ns[s])
        if s % 2 == 0:
            if s % 4 == 0:
                nx = max(2, int(round(np.sqrt(n))))
                ny = max(2, int(round(n / nx)))
                mats.append(poisson2d(nx, ny))
                kinds.append("poisson2d")
            else:
                nx = max(2, int(round(n ** (1.0 / 3.0))))
                nz = max(2, int(round(n / (nx * nx))))
                mats.append(poisson3d(nx, nx, nz))
                kinds.append("poisson3d")
        else:
            r = np.random.default_rng([seed, s])
            m = int(r.integers(4, 14))
            offs = r.choice(np.arange(1, n // 2), size=m, replace=False)
            w = 1.0 - r.uniform(0.0, 0.9, m)  # in (0.1, 1]
            mats.append(circulant_laplacian(n, np.sort(offs), w, shift=1e-3))
            kinds.append("circulant")
    A = CSR.from_scipy(sp.block_diag([m.to_scipy() for m in mats], format="csr"))
    off = np.zeros(nsys + 1, dtype=np.int64)
    off[1:] = np.cumsum([m.n for m in mats])
    xt = np.concatenate([uniform(m.n, 4000 + s) for s, m in enumerate(mats)])
    b = A.matvec(xt)
    return Batch(A=A, sys_row_off=off.astype(np.int32), b=b, x_true=xt, kinds=kinds)


@dataclass
class AdjointProblem:
    """A(theta) = 7-point Laplacian + diag(theta); loss 0.5 ||x - x_target||^2."""
    lap: CSR           # the Laplacian alone
    theta: np.ndarray
    b: np.ndarray
    x_target: np.ndarray
    diag_pos: np.ndarray  # index into val of every diagonal entry

    def matrix(self, theta=None):
        th = self.theta if theta is None else np.asarray(theta, dtype=np.float64)
        val = self.lap.val.copy()
        val[self.diag_pos] += th
        return CSR(n=self.lap.n, row_ptr=self.lap.row_ptr, col_idx=self.lap.col_idx, val=val)


def diagonal_positions(A):
    """Index in A.val of each row's diagonal entry (every row must have one)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    pos = np.nonzero(A.col_idx == rows)[0]
    if pos.size != A.n:
        raise ValueError("matrix lacks a full diagonal")
    return pos


def adjoint_problem(nx=100, seed=5, bseed=555, tseed=55):
    """theta ~ U[0.01, 1] (seed), b ~ U[-1, 1] (bseed), x_target ~ N(0, 1) (tseed)."""
    lap = poisson3d(nx)
    theta = np.random.default_rng(seed).uniform(0.01, 1.0, lap.n)
    b = uniform(lap.n, bseed)
    xt = np.random.default_rng(tseed).standard_normal(lap.n)
    return AdjointProblem(lap=lap, theta=theta, b=b, x_target=xt, diag_pos=diagonal_positions(lap))
