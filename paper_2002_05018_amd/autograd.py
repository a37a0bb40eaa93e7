"""torch.autograd.Function whose backward pass is the adjoint solve.

Forward: eps_r -> (reassemble A_d, factor, solve) -> E = S(eps_r)^{-1} f.
Backward: S is complex symmetric, so the adjoint system reuses the same
factors: w = S^{-1} conj(G) with G = dL/dRe E + j dL/dIm E (PyTorch's
convention for complex outputs), and dL/d eps_r,t = k^2 Re sum_rhs
w_t^T M_t E_t (M_t the unit-eps_r element mass), computed by d3m_adjoint.
The gradient with respect to the load f is conj(w).

The handle holds one set of factors.  When it has been refactored since this
forward (another forward, a finite-difference probe, a line search), the
backward first restores the factors of this forward's eps_r (update_eps and
factor with the same precision), so the adjoint always solves with S of the
eps_r that produced E; the handle then keeps those factors.
"""
import torch


class D3MSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, solver, rhs, precision=0):
        eps = eps_r.detach().cpu().double().numpy().copy()
        solver.update_eps(eps)
        solver.factor(precision)
        E = solver.solve(rhs.detach())
        ctx.solver = solver
        ctx.eps = eps
        ctx.precision = precision
        ctx.generation = solver.generation
        ctx.eps_device = eps_r.device
        ctx.save_for_backward(E)
        ctx.rhs_requires_grad = rhs.requires_grad
        return E

    @staticmethod
    def backward(ctx, grad_E):
        (E,) = ctx.saved_tensors
        solver = ctx.solver
        if solver.generation != ctx.generation:
            solver.update_eps(ctx.eps)
            solver.factor(ctx.precision)
            ctx.generation = solver.generation
        grad_eps, w = solver.adjoint(grad_E.contiguous(), E, want_w=True)
        grad_rhs = torch.conj(w) if ctx.rhs_requires_grad else None
        return grad_eps.to(device=ctx.eps_device, dtype=torch.float64), None, grad_rhs, None
