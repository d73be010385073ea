"""Differentiable MAS-PCG solve: x = H^-1 b as a torch.autograd.Function.

Backward solves the adjoint system H lambda = dL/dx with the forward MAS
preconditioner (H is symmetric, so the preconditioner built for the forward
system also serves the adjoint one) and returns dL/db = lambda and
dL/dH_ij = -lambda_i x_j^T on every stored block (from dx = -H^-1 (dH) x).
Both the solve and the scatter run in the library's HIP kernels.

Neither solve may stop at max_iter: a forward solve that does not reach tol
raises MasError (x would not be H^-1 b), and so does an adjoint solve that
does not (lambda, dL/db and dL/dH would not be the gradient).
"""

import torch

from .solver import BlockMatrix


class MasPcgSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, b, solver, row_ptr, col_idx, tol, max_iter, rebuild):
        H = BlockMatrix(row_ptr, col_idx, val.detach())
        if rebuild:
            solver.build(H)
        x, res = solver.solve(H, b.detach(), tol=tol, max_iter=max_iter, allow_not_converged=False)
        ctx.solver = solver
        ctx.tol = tol
        ctx.max_iter = max_iter
        ctx.result = res
        ctx.save_for_backward(val, x, row_ptr, col_idx)
        return x

    @staticmethod
    def backward(ctx, dx):
        val, x, row_ptr, col_idx = ctx.saved_tensors
        H = BlockMatrix(row_ptr, col_idx, val.detach())
        lam, dH, res = ctx.solver.adjoint(
            H,
            x,
            dx.contiguous().to(torch.float64),
            dLdH_dtype=val.dtype,
            want_dH=ctx.needs_input_grad[0],
            tol=ctx.tol,
            max_iter=ctx.max_iter,
            allow_not_converged=False,
        )
        ctx.adjoint_result = res
        dval = dH.view_as(val) if dH is not None else None
        db = lam if ctx.needs_input_grad[1] else None
        return dval, db, None, None, None, None, None, None


def mas_pcg_solve(solver, H, b, tol=1e-6, max_iter=10000, rebuild=True):
    """x = H^-1 b, differentiable w.r.t. ``H.val`` and ``b``."""
    return MasPcgSolve.apply(H.val, b, solver, H.row_ptr, H.col_idx, tol, max_iter, rebuild)
