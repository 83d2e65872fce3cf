"""Differentiable quantity of interest Q(theta0, s_1..s_M) of the SG solution.

Forward: solve the SG system with the preconditioned flexible CG and evaluate
Q = w_mean . E[u] + w_var . Var[u] on the device. Backward: the hand-written
adjoint in the library (sg_adjoint_grad) solves A Lambda = dQ/dU with the
same preconditioner and contracts -<Lambda, (dA/dtheta) U>.
"""

from __future__ import annotations

import copy
from dataclasses import dataclass, field

import numpy as np
import torch

from .binding import Options, SGSolver


@dataclass
class QoISpec:
    problem: object          # n_e, M, p, sigma, phi (theta0 and s are replaced by theta)
    F: torch.Tensor          # (P, n) right-hand side on the device
    w_mean: torch.Tensor     # (n,) device
    w_var: torch.Tensor      # (n,) device
    opts: Options = field(default_factory=Options)
    rtol: float = 1e-8
    maxit: int = 200
    last_stats: dict = field(default_factory=dict)


class SGQoI(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, spec: QoISpec):
        th = theta.detach().to("cpu", torch.float64).numpy()
        prob = copy.copy(spec.problem)
        prob.theta0 = float(th[0])
        prob.s = np.array(th[1:], dtype=np.float64)
        solver = SGSolver(prob, spec.opts, device=spec.F.device)
        U, st = solver.sg_solve(spec.F, rtol=spec.rtol, maxit=spec.maxit)
        spec.last_stats = {"forward": st}
        Q = solver.sg_qoi(U, spec.w_mean, spec.w_var)
        ctx.solver, ctx.U, ctx.spec = solver, U, spec
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return torch.tensor(Q, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, gQ):
        spec = ctx.spec
        if ctx.solver is None:
            raise RuntimeError("SGQoI: backward ran already; the handle is released after the first backward")
        try:
            _, grad, st = ctx.solver.sg_adjoint_grad(ctx.U, spec.w_mean, spec.w_var, rtol=spec.rtol,
                                                     maxit=spec.maxit)
        finally:
            ctx.solver.close()
            ctx.solver = None
        spec.last_stats["adjoint"] = st
        g = torch.from_numpy(grad).to(ctx.theta_device, ctx.theta_dtype)
        return gQ * g, None
