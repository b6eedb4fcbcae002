"""Differentiable multi-word CG solve (torch.autograd.Function).

Forward: x = A^-1 b by the library's CG in the chosen arithmetic (Alg. 1),
returned rounded to FP64.  Backward: lam = A^-T g (g = dL/dx) by the same
CG (A is SPD, so A^T = A); dL/db = lam; dL/dA_ij = -lam_i x_j on A's
pattern (mw_csr_grad).  Gradients reach any parameter the values depend
on through ordinary autograd (e.g. dL/dtheta_i = -lam_i x_i for
A = L + diag(theta)).  Every step runs in libmwcg; this module only wires
the calls into autograd.  MWCGSolveBatched does the same for many
independent systems on the diagonal blocks of one matrix: one batched
forward solve, one batched adjoint solve, and the gradient on the whole
block-diagonal pattern.  The mixed-precision arithmetics (MXDW, MXQTW)
keep x and lam in FP64: their rounding to FP64 is the identity, and the
product lam_i x_j rounded once to FP64 is the FP64 product, so those two
steps take the FP64 entry points.
"""
import torch

from . import mw


def _vector_arith(arith):
    """The arithmetic of the stored vectors: FP64 for the mixed types."""
    return "fp64" if mw.WORDS[arith] == 1 else arith


class MWCGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, b, row_ptr, col_idx, arith, tol, maxit, info_out, precond=None):
        A = mw.DeviceCSR(b.numel(), row_ptr, col_idx, val.detach().contiguous())
        # one SpMV plan (the solver's own choice) and workspace serve the
        # forward and the adjoint solve
        plan = mw.Plan(A, solver=arith)
        ws = mw.cg_workspace(arith, A)
        x, info = mw.cg_solve(arith, A, b.detach().contiguous(), tol=tol, maxit=maxit, plan=plan, workspace=ws,
                              precond=precond)
        if info["status"] != "ok":
            raise mw.MWError("forward solve did not converge: %s" % info)
        ctx.A, ctx.arith, ctx.tol, ctx.maxit, ctx.info_out = A, arith, tol, maxit, info_out
        ctx.precond = precond
        ctx.plan, ctx.ws = plan, ws
        ctx.x = x
        if info_out is not None:
            info_out["forward"] = info
        return mw.elementwise(_vector_arith(arith), "tofp64", x).reshape(-1)

    @staticmethod
    def backward(ctx, grad_x):
        A, arith = ctx.A, ctx.arith
        lam, info = mw.cg_solve(arith, A, grad_x.detach().contiguous().reshape(-1), tol=ctx.tol, maxit=ctx.maxit,
                                plan=ctx.plan, workspace=ctx.ws, precond=ctx.precond)
        if info["status"] != "ok":
            raise mw.MWError("adjoint solve did not converge: %s" % info)
        if ctx.info_out is not None:
            ctx.info_out["adjoint"] = info
            ctx.info_out["lam"] = lam
            ctx.info_out["x"] = ctx.x
        va = _vector_arith(arith)
        grad_b = mw.elementwise(va, "tofp64", lam).reshape(-1)
        grad_val = mw.csr_grad(va, A, lam, ctx.x)
        return grad_val, grad_b, None, None, None, None, None, None, None


def cg_solve(A, val, b, arith="qtw", tol=1e-12, maxit=None, info=None, precond=None):
    """x = A(val)^-1 b, differentiable in val and b.  A supplies n, row_ptr
    and col_idx (a DeviceCSR); val: FP64 values on A's pattern.  precond:
    None or "jacobi", for the forward and the adjoint solve alike (it
    changes how the solves get there, not the gradient's formula)."""
    if maxit is None:
        maxit = min(10 * A.n, mw.MAXIT_MAX)
    return MWCGSolve.apply(val, b, A.row_ptr, A.col_idx, arith, tol, maxit, info, precond)


class MWCGSolveBatched(torch.autograd.Function):
    """x_s = A_s^-1 b_s for the systems on A's diagonal blocks (rows
    sys_row_off[s] .. sys_row_off[s+1]-1), by one batched solve forward
    and one batched adjoint solve backward; per system the same formulas
    as MWCGSolve."""

    @staticmethod
    def forward(ctx, val, b, row_ptr, col_idx, sys_row_off, arith, tol, maxit, info_out, precond=None):
        A = mw.DeviceCSR(b.numel(), row_ptr, col_idx, val.detach().contiguous())
        nbytes = mw.lib().mw_cg_batched_workspace_bytes(mw.ARITH[arith], len(sys_row_off) - 1, A.n, A.nnz)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
        x, iters, status, rel, info = mw.cg_solve_batched(arith, A, sys_row_off, b.detach().contiguous(), tol=tol,
                                                          maxit=maxit, workspace=ws, precond=precond)
        if (status != 0).any():
            raise mw.MWError("forward solve of systems %s did not converge" % list((status != 0).nonzero()[0]))
        ctx.A, ctx.off, ctx.arith, ctx.tol, ctx.maxit, ctx.info_out = A, sys_row_off, arith, tol, maxit, info_out
        ctx.precond, ctx.ws, ctx.x = precond, ws, x
        if info_out is not None:
            # per-system arrays, and the batch's summary under "batch"
            info_out["forward"] = {"iters": iters, "status": status, "rel_res": rel, "batch": info}
        return mw.elementwise(_vector_arith(arith), "tofp64", x).reshape(-1)

    @staticmethod
    def backward(ctx, grad_x):
        A, arith = ctx.A, ctx.arith
        lam, iters, status, rel, info = mw.cg_solve_batched(arith, A, ctx.off, grad_x.detach().contiguous().reshape(-1),
                                                            tol=ctx.tol, maxit=ctx.maxit, workspace=ctx.ws,
                                                            precond=ctx.precond)
        if (status != 0).any():
            raise mw.MWError("adjoint solve of systems %s did not converge" % list((status != 0).nonzero()[0]))
        if ctx.info_out is not None:
            ctx.info_out["adjoint"] = {"iters": iters, "status": status, "rel_res": rel, "batch": info}
        va = _vector_arith(arith)
        grad_b = mw.elementwise(va, "tofp64", lam).reshape(-1)
        grad_val = mw.csr_grad(va, A, lam, ctx.x)
        return grad_val, grad_b, None, None, None, None, None, None, None, None


def cg_solve_batched(A, val, sys_row_off, b, arith="qtw", tol=1e-12, maxit=None, info=None, precond=None):
    """x = A(val)^-1 b for the independent systems on A's diagonal blocks
    (sys_row_off: host sequence of nsys + 1 row offsets), differentiable in
    val and b, all systems in one batched forward and one batched adjoint
    solve.  Other arguments as cg_solve; maxit None: 10 x the largest
    system's rows."""
    import numpy as np
    off = np.ascontiguousarray(np.asarray(sys_row_off, dtype=np.int32))
    if maxit is None:
        maxit = min(10 * int(np.max(np.diff(off))), mw.MAXIT_MAX)
    return MWCGSolveBatched.apply(val, b, A.row_ptr, A.col_idx, off, arith, tol, maxit, info, precond)
