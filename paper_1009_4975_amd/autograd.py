"""Compliance as a differentiable function of the element densities.

forward(rho) = c(rho) = f^T u with K(rho) u = f (paper Sec. 3, Eq. (1)), solved
by the library's PCG.  Compliance is self-adjoint (the adjoint state is -u), so
backward needs no second solve: dc/drho_e = -p rho_e^(p-1) (E0 - Emin) h_e
u_e^T K0 u_e, evaluated by the library's sensitivity kernel on the saved u.
"""
from __future__ import annotations

import torch

from . import binding


class ComplianceProblem:
    """A mesh, its load and solver settings on one device context."""

    def __init__(self, mesh: "binding.MeshArrays", rtol=1e-10, inner_prec=binding.FP64, inner_rtol=0.1,
                 max_it=100000, device=0):
        self.ctx = binding.Context(device)
        self.ctx.upload_mesh(mesh)
        self.mesh = mesh
        self.f = torch.tensor(mesh.f_load, dtype=torch.float64, device="cuda")
        self.b = torch.empty_like(self.f)
        self.ctx.project_rhs(self.f, self.b)
        self.rtol, self.inner_prec, self.inner_rtol, self.max_it = rtol, inner_prec, inner_rtol, max_it
        self.u = torch.zeros_like(self.f)  # warm start across calls (paper Sec. 5)
        self.last_stats = None

    def solve(self, rho: torch.Tensor) -> torch.Tensor:
        self.ctx.set_density(rho)
        u = self.u.clone()
        self.last_stats = self.ctx.pcg(self.b, u, rtol=self.rtol, max_it=self.max_it, inner_prec=self.inner_prec,
                                       inner_rtol=self.inner_rtol)
        self.u = u
        return u


class ComplianceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho: torch.Tensor, problem: ComplianceProblem):
        rho = rho.detach().contiguous()
        u = problem.solve(rho)
        c = problem.ctx.compliance(u, problem.f)
        ctx.save_for_backward(rho, u)
        ctx.problem = problem
        return torch.tensor(c, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_c):
        rho, u = ctx.saved_tensors
        dc = torch.empty_like(rho)
        ctx.problem.ctx.sensitivity(u, rho, dc)
        return grad_c * dc, None


def compliance(rho: torch.Tensor, problem: ComplianceProblem) -> torch.Tensor:
    return ComplianceFn.apply(rho, problem)
