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

import math

import torch

from . import dse as _dse


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


def chebyshev_basis(solver: "_dse.Solver", points, which: str = "Z") -> torch.Tensor:
    """Matrix B[m, j] = Tilde-T_j(s(p_m)) (Sec. 3 expansion, c_0/2 convention)
    so that ln Z(p_m) = B @ a (or ln G(p_m) = B @ b) for points inside
    [eps2, lambda2]."""
    p = solver.p
    n = p.n_z if which == "Z" else p.n_g
    x = torch.as_tensor(points, dtype=torch.float64, device=solver.device)
    L0 = 0.5 * (math.log(p.eps2) + math.log(p.lambda2))
    L1 = 0.5 * (math.log(p.lambda2) - math.log(p.eps2))
    s = ((torch.log(x) - L0) / L1).clamp(-1.0, 1.0)
    cols = [torch.ones_like(s), s]  # T_0, T_1; the recurrence needs T_0 = 1
    for _ in range(2, n):
        cols.append(2.0 * s * cols[-1] - cols[-2])
    cols[0] = torch.full_like(s, 0.5)  # Tilde-T_0 = 1/2
    return torch.stack(cols[:n], dim=1)
