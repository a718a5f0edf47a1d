"""Differentiable u(T) = U_{L,M}(u0, nu) through the HIP adjoint sweep.

Forward: aao_solve of C(nu) U = w(u0) (eq. (globalsys)).  Backward: the
transposed all-at-once system C^T lambda = e_{L,M} (x) g solved by the same
alpha-circulant machinery (aao_adjoint_solve), then aao_grad gives
dJ/du0 = sum_m lambda_{1,m} and dJ/dnu = dT sum_l lambda_l^T (Q (x) dA/dnu) U_l.
"""
import torch

from .stencil import plan_for, taps_for

_PLANS = {}


def _plan(workload, nu):
    """One plan per workload shape; nu only changes the stencil weights
    (aao_set_stencil_coef), so a new nu does not re-plan."""
    key = workload.with_(nu=0.0)
    p = _PLANS.get(key)
    if p is None:
        if len(_PLANS) > 8:
            _PLANS.clear()
        p = plan_for(workload.with_(nu=float(nu)))
        _PLANS[key] = p
    w = workload
    _, _, coef, dcoef = taps_for(w.kind, w.nx, w.ny, nu=float(nu), vel=w.vel, order=w.order)
    p.set_stencil_coef(coef, dcoef)
    return p, coef, dcoef


class AAOSolve(torch.autograd.Function):
    """u(T) [B, N] from u0 [B, N] (float64, cuda) and a scalar nu tensor."""

    @staticmethod
    def forward(ctx, u0, nu, workload, tol, adj_tol, max_iter):
        plan, coef, dcoef = _plan(workload, nu.item())
        plan.set_u0(u0.detach())
        u, info = plan.solve(tol=tol, stop=workload.stop, max_iter=max_iter,
                             alphas=[workload.alpha] if workload.alpha > 0 else None)
        ctx.plan = plan
        ctx.coef, ctx.dcoef = coef, dcoef
        ctx.u = u
        ctx.adj_tol = adj_tol
        ctx.max_iter = max_iter
        ctx.info = info
        ctx.nu_shape = nu.shape
        return u[:, -1, -1, :].clone()

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        plan.set_stencil_coef(ctx.coef, ctx.dcoef)  # another forward may have changed nu
        lam, _ = plan.adjoint_solve(g.detach().to(torch.float64).contiguous(), tol=ctx.adj_tol,
                                    max_iter=ctx.max_iter)
        gu0, gnu = plan.grad(ctx.u, lam)
        return gu0, gnu.sum().reshape(ctx.nu_shape), None, None, None, None


def solve_uT(u0, nu, workload, tol=None, adj_tol=None, max_iter=50):
    """Differentiable U_{L,M}; nu is a 0-d float64 tensor (requires_grad allowed)."""
    tol = workload.tol if tol is None else tol
    adj_tol = tol if adj_tol is None else adj_tol
    return AAOSolve.apply(u0, nu, workload, tol, adj_tol, max_iter)
