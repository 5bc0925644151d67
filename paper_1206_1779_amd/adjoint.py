"""Differentiating the converged dressings with respect to the physical
parameters theta = (alpha(mu^2), G(x_G)^{-1}, Z(x_Z)^{-1}).

The Newton root c*(theta) satisfies F(c*, theta) = 0, so by the implicit
function theorem dc*/dtheta = -J^{-1} dF/dtheta with J = dF/dc at the root.
For a scalar loss L(c*) the backward pass needs one transposed solve,
J^T lambda = dL/dc, and one parameter vector-Jacobian product,
dL/dtheta = -lambda^T dF/dtheta: both run in the HIP library
(dse_lu_solve with trans = 1, dse_vjp).  This module only wires them into
torch.autograd.
"""
from __future__ import annotations

import torch


class ImplicitSolve(torch.autograd.Function):
    """c* = ImplicitSolve.apply(theta, solver, c0, newton_kwargs).

    theta: float64 tensor (alpha_mu, g0_inv, z_lambda_inv); solver: a
    dse.Solver whose grid defines the discretisation; c0: start (None = the
    asymptotic start guess)."""

    @staticmethod
    def forward(ctx, theta, solver, c0, newton_kwargs):
        a, g, z = (float(x) for x in theta.detach().cpu())
        solver.set_physics(a, g, z)
        res = solver.newton(c0, **(newton_kwargs or {}))
        ctx.solver = solver
        ctx.theta = (a, g, z)
        ctx.theta_device = theta.device
        ctx.save_for_backward(res.c)
        return res.c

    @staticmethod
    def backward(ctx, grad_c):
        (c,) = ctx.saved_tensors
        s = ctx.solver
        s.set_physics(*ctx.theta)
        J = s.jacobian(c, with_F=False)
        lam = s.lu_solve(J, grad_c.detach().to(torch.float64).contiguous(), trans=True)
        _, ut = s.vjp(c, lam, with_c=False)
        return -ut.to(ctx.theta_device), None, None, None


class DressingsAt(torch.autograd.Function):
    """(ln Z(u), ln G(u)) = DressingsAt.apply(c, solver, u): the dressings at
    momenta u from the coefficients c (dse_running_coupling), differentiable in
    c through dse_dressing_vjp (d ln Z(u)/d a_j = d ln G(u)/d b_j =
    Tilde-T_j(s(u)), Sec. 3 expansion).  Both directions run in the HIP
    library; this class only wires them into torch.autograd."""

    @staticmethod
    def forward(ctx, c, solver, u):
        u = torch.as_tensor(u, dtype=torch.float64).to(solver.device).contiguous().reshape(-1)
        _, lnz, lng = solver.running_coupling(c.detach(), u)
        ctx.solver = solver
        ctx.save_for_backward(u)
        return lnz, lng

    @staticmethod
    def backward(ctx, g_lnz, g_lng):
        (u,) = ctx.saved_tensors
        gc = ctx.solver.dressing_vjp(u, g_lnz, g_lng)
        return gc, None, None
