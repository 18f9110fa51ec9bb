"""Differentiable seeded solve: a torch.autograd.Function around the C ABI.

Forward: x_j = A^{-1} b_j for A = D^H D by the single-seed method (seed on
b_1, project the others over the Lanczos basis, finish with CG).
Backward, for the incoming gradient g_j = dL/dRe x_j + i dL/dIm x_j (PyTorch's
convention for complex tensors and a real loss): the adjoint systems
A lambda_j = g_j are extra right-hand sides of the same Hermitian A, so they
are projected over the forward basis and finished with CG; then
    dL/db_j   = lambda_j,
    dL/dkappa = sum_j Re[(H lambda_j)^H D x_j + (D lambda_j)^H H x_j],
with D = 1 - kappa H, so dA/dkappa = -(H^H D + D^H H).  Every step runs in the
HIP library; this module only passes tensors through.
"""
import torch

from . import api


class SeededSolve(torch.autograd.Function):
    """X = SeededSolve.apply(B, kappa, U, dims, m, freq, tol, antiperiodic, mixed).

    B: (k, n) complex128 right-hand sides in the library field layout, on the GPU.
    kappa: 0-d float64 tensor (may require grad).  U: links in the library layout.
    """

    @staticmethod
    def forward(ctx, B, kappa, U, dims, m, freq, tol, antiperiodic=True, mixed=False):
        op = api.Op.wilson(dims, U, float(kappa), antiperiodic, single=True)
        out = api.seeded_solve(op, B.detach(), m, freq, tol, mixed=mixed)
        ctx.op = op
        ctx.basis = out["basis"]
        ctx.tol = tol
        ctx.mixed = mixed
        ctx.stats = {"iters": out["iters"], "relres": out["relres"]}
        ctx.save_for_backward(out["X"])
        return out["X"]

    @staticmethod
    def backward(ctx, grad_X):
        (X,) = ctx.saved_tensors
        op = ctx.op
        G = grad_X.detach().to(torch.complex128).contiguous()
        # adjoint right-hand sides seeded from the forward Lanczos basis
        Lam0 = api.project(ctx.basis, G)
        Lam, its, rel = api.solve_cg(op, G, ctx.tol, X0=Lam0, mixed=ctx.mixed)
        ctx.stats["adjoint_iters"] = its
        grad_B = Lam if ctx.needs_input_grad[0] else None
        grad_k = None
        if ctx.needs_input_grad[1]:
            grad_k = torch.tensor(op.kappa_grad(X, Lam), dtype=torch.float64, device=X.device)
        return grad_B, grad_k, None, None, None, None, None, None, None


def seeded_solve(B, kappa, U, dims, m, freq, tol, antiperiodic=True, mixed=False):
    return SeededSolve.apply(B, kappa, U, dims, m, freq, tol, antiperiodic, mixed)
