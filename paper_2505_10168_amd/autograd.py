"""Differentiable time-integrated thermal compliance (Section 7).

``ThermalCompliance.apply(rho, solver)`` returns Theta = b^T u dt / Theta_ref
(Section 7.1) for the element densities ``rho`` on a device-resident STMG hierarchy;
its backward pass is the gradient g_e = -Lambda^T (dJ/drho_e) u with Lambda from the
adjoint system J^T Lambda = b dt / Theta_ref (Section 7.2), all in libstmg.  PyTorch
only carries the tensors and the autograd graph.

The adjoint right-hand side does not depend on u, so by default the forward pass also
solves the adjoint system, concurrently, on a second handle with its own stream (the
latency-bound coarse levels of one solve overlap the other's work); backward then only
forms the gradient.  With ``concurrent_adjoint=False`` the adjoint is solved in
backward, on the same handle.  With ``warm_start=True`` each solve starts from the
previous design's solution instead of zero (a design loop changes the design a little
per step, so fewer V-cycles reach the tolerance).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import torch

from . import binding as B

_STATUS = {B.STMG_OK: "ok", B.STMG_NOT_CONVERGED: "not converged", B.STMG_DIVERGED: "diverged"}


def _check(st, what, strict):
    if st.status != B.STMG_OK and strict:
        raise RuntimeError(f"{what} STMG solve {_STATUS.get(st.status, st.status)}: "
                           f"relative residual {st.rel_residual:.3e} after {st.cycles} cycles")


class ThermalCompliance(torch.autograd.Function):
    """Theta(rho) with an STMG forward solve and an STMG adjoint backward."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, solver: "ComplianceSolver") -> torch.Tensor:
        rho = rho.detach().to(torch.float64).contiguous()
        version = solver._load_design(rho)
        pending = solver._start_adjoint() if solver.concurrent else None
        u, st = solver.solver.solve_forward(u0=solver._u_prev if solver.warm_start else None)
        solver.last_forward = st
        if solver.warm_start:
            solver._u_prev = u
        lam = None
        if pending is not None:
            lam, sa = pending.result()
            solver.last_adjoint = sa
            _check(sa, "adjoint", solver.strict)
        _check(st, "forward", solver.strict)
        theta = solver.solver.objective(u)
        ctx.solver = solver
        ctx.version = version
        ctx.save_for_backward(rho, u, lam if lam is not None else u.new_empty(0))
        ctx.has_lam = lam is not None
        return torch.tensor(theta, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        rho, u, lam = ctx.saved_tensors
        solver = ctx.solver
        if solver.version != ctx.version:
            solver._load_design(rho)
        if not ctx.has_lam:
            lam, st = solver.solver.solve_adjoint(
                l0=solver._lam_prev if solver.warm_start else None)
            solver.last_adjoint = st
            _check(st, "adjoint", solver.strict)
            if solver.warm_start:
                solver._lam_prev = lam
        g = solver.solver.gradient(u, lam)
        return grad_out * g, None


class ComplianceSolver:
    """Owns the STMG hierarchy (two, with the concurrent adjoint) for a fixed grid and
    material; designs are loaded into it by re-assembly.  deff_mode = 1 (Section 7.2)
    keeps the coarsening path fixed across designs, so the hierarchy never needs to be
    rebuilt."""

    def __init__(self, problem: B.Problem, rho0: torch.Tensor, q: torch.Tensor | None = None,
                 strict: bool = True, concurrent_adjoint: bool = True,
                 warm_start: bool = False, **options):
        options.setdefault("deff_mode", 1)
        rho0 = rho0.detach().to(torch.float64).contiguous()
        self.concurrent = concurrent_adjoint
        dev = rho0.device
        s1 = torch.cuda.Stream(device=dev) if concurrent_adjoint else None
        s2 = torch.cuda.Stream(device=dev) if concurrent_adjoint else None
        self.solver = B.Solver(problem, rho0, q=q, stream=s1, **options)
        self.adjoint_solver = (B.Solver(problem, rho0, q=q, stream=s2, **options)
                               if concurrent_adjoint else None)
        self._pool = ThreadPoolExecutor(max_workers=1) if concurrent_adjoint else None
        self.version = 0
        self._current = rho0.clone()
        self.strict = strict
        self.warm_start = warm_start
        self._u_prev = None
        self._lam_prev = None
        self.last_forward = None
        self.last_adjoint = None

    def _load_design(self, rho: torch.Tensor) -> int:
        if not (self._current.shape == rho.shape and torch.equal(self._current, rho)):
            self.solver.set_design(rho)
            if self.adjoint_solver is not None:
                self.adjoint_solver.set_design(rho)
            self._current = rho.clone()
            self.version += 1
        return self.version

    def _start_adjoint(self):
        def run():
            lam, st = self.adjoint_solver.solve_adjoint(
                l0=self._lam_prev if self.warm_start else None)
            if self.warm_start:
                self._lam_prev = lam
            return lam, st
        return self._pool.submit(run)

    def __call__(self, rho: torch.Tensor) -> torch.Tensor:
        return ThermalCompliance.apply(rho, self)

    def close(self):
        self.solver.close()
        if self.adjoint_solver is not None:
            self.adjoint_solver.close()
            self._pool.shutdown()
