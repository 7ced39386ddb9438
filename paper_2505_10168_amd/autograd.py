"""Differentiable time-integrated thermal compliance (Section 7).

``ThermalCompliance.apply(rho, solver)`` returns Theta = b^T u dt / Theta_ref
(Section 7.1) for the element densities ``rho`` on a device-resident STMG hierarchy;
its backward pass is the adjoint STMG solve J^T Lambda = b dt / Theta_ref (Section
7.2) followed by the gradient kernel g_e = -Lambda^T (dJ/drho_e) u, all in libstmg.
PyTorch only carries the tensors and the autograd graph.
"""
from __future__ import annotations

import torch

from . import binding as B

_STATUS = {B.STMG_OK: "ok", B.STMG_NOT_CONVERGED: "not converged", B.STMG_DIVERGED: "diverged"}


class ThermalCompliance(torch.autograd.Function):
    """Theta(rho) with an STMG forward solve and an STMG adjoint backward."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, solver: "ComplianceSolver") -> torch.Tensor:
        rho = rho.detach().to(torch.float64).contiguous()
        version = solver._load_design(rho)
        u, st = solver.solver.solve_forward()
        solver.last_forward = st
        if st.status != B.STMG_OK and solver.strict:
            raise RuntimeError(f"forward STMG solve {_STATUS.get(st.status, st.status)}: "
                               f"relative residual {st.rel_residual:.3e} after {st.cycles} cycles")
        theta = solver.solver.objective(u)
        ctx.solver = solver
        ctx.version = version
        ctx.save_for_backward(rho, u)
        return torch.tensor(theta, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        rho, u = ctx.saved_tensors
        solver = ctx.solver
        if solver.version != ctx.version:
            solver._load_design(rho)
        lam, st = solver.solver.solve_adjoint()
        solver.last_adjoint = st
        if st.status != B.STMG_OK and solver.strict:
            raise RuntimeError(f"adjoint STMG solve {_STATUS.get(st.status, st.status)}: "
                               f"relative residual {st.rel_residual:.3e} after {st.cycles} cycles")
        g = solver.solver.gradient(u, lam)
        return grad_out * g, None


class ComplianceSolver:
    """Owns one STMG hierarchy for a fixed grid and material; designs are loaded into
    it by re-assembly.  deff_mode = 1 (Section 7.2) keeps the coarsening path fixed
    across designs, so the hierarchy never needs to be rebuilt."""

    def __init__(self, problem: B.Problem, rho0: torch.Tensor, strict: bool = True, **options):
        options.setdefault("deff_mode", 1)
        self.solver = B.Solver(problem, rho0.detach().to(torch.float64).contiguous(), **options)
        self.version = 0
        self._current = rho0.detach().clone()
        self.strict = strict
        self.last_forward = None
        self.last_adjoint = None

    def _load_design(self, rho: torch.Tensor) -> int:
        if not (self._current.shape == rho.shape and torch.equal(self._current, rho)):
            self.solver.set_design(rho)
            self._current = rho.clone()
            self.version += 1
        return self.version

    def __call__(self, rho: torch.Tensor) -> torch.Tensor:
        return ThermalCompliance.apply(rho, self)

    def close(self):
        self.solver.close()
