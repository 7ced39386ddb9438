"""Design loop of the optimisation problem of Section 7 on one resident STMG hierarchy.

Every optimisation cycle evaluates Theta(rho) and dTheta/drho through
``ComplianceSolver`` (forward and adjoint STMG solves, concurrent, in libstmg; the
field-independent coarsening path of Section 7.2, so a new design only re-assembles
the levels; optionally warm restarts from the previous cycle's u and Lambda) and then
moves the design with ``stmg_oc_update``, the optimality-criteria step for the box and
volume constraints of Section 7.1 (the paper's MMA is only cited there).  The loop
stops by the rule of Section 7.2: the relative change of Theta stays below 0.1 % for
5 consecutive cycles.  Python only sequences the library calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from . import inputs
from .autograd import ComplianceSolver

# Solver settings of the optimisation study (Section 7.2): six levels, lambda_crit =
# 0.25, 20 smoothing steps, the field-independent D_eff of the SIMP extremes.
SECTION7_OPTIONS = dict(max_levels=6, lambda_crit=0.25, nu=20, deff_mode=1,
                        reassembly=B.STMG_REASSEMBLE_R)


def section7_problem(n_el: int = 256, n_t: int = 256) -> tuple[B.Problem, np.ndarray]:
    """The optimisation problem of Section 7.1: problem 7's rod (L = 0.1 m, t_T = 10 s,
    aluminium / epoxy of the material table, p_k = 3, p_c = 2), the many-frequency
    heat load of Section 3.1 and Theta_ref = 1e6.  Returns the problem and the load
    (shape (n_t + 1, n_el), row 0 unused)."""
    prob = B.Problem(n_el, n_t, length=0.1, t_final=10.0, k_ins=0.197, k_con=214.0,
                     c_ins=1.67e6, c_con=2.41e6, p_k=3.0, p_c=2.0, theta_ref=1e6)
    return prob, inputs.paper_heat_load(n_el, n_t, 0.1, 10.0)


@dataclass
class DesignHistory:
    theta: list = field(default_factory=list)
    volume: list = field(default_factory=list)
    forward_cycles: list = field(default_factory=list)
    adjoint_cycles: list = field(default_factory=list)
    dof_updates: float = 0.0
    converged: bool = False


class DesignLoop:
    """Minimise Theta(rho) subject to 0 <= rho <= 1 and mean(rho) <= volume."""

    def __init__(self, problem: B.Problem, rho0: torch.Tensor, volume: float = 0.5,
                 q: torch.Tensor | None = None, move: float = 0.2, eta: float = 0.5,
                 rho_min: float = 1e-3, warm_start: bool = True, rtol: float = 1e-3,
                 patience: int = 5, keep_designs: bool = False, **options):
        self.volume, self.move, self.eta, self.rho_min = volume, move, eta, rho_min
        self.rtol, self.patience = rtol, patience
        self.rho = rho0.detach().to(torch.float64).contiguous().clone()
        self.compliance = ComplianceSolver(problem, self.rho, q=q, warm_start=warm_start,
                                           **options)
        self.history = DesignHistory()
        self.designs = [] if keep_designs else None
        self.last_gradient = None
        self._calm = 0

    def step(self) -> float:
        """One optimisation cycle: Theta and its gradient at the current design, then
        the design update (skipped once the stopping rule holds).  Returns Theta of the
        design it started from."""
        x = self.rho.clone().requires_grad_(True)
        theta = self.compliance(x)
        theta.backward()
        g = x.grad.detach()
        h = self.history
        if self.designs is not None:
            self.designs.append(self.rho.clone())
        h.theta.append(float(theta.detach()))
        h.volume.append(float(self.rho.mean()))
        h.forward_cycles.append(self.compliance.last_forward.cycles)
        h.adjoint_cycles.append(self.compliance.last_adjoint.cycles)
        h.dof_updates += (self.compliance.last_forward.dof_updates +
                          self.compliance.last_adjoint.dof_updates)
        self.last_gradient = g
        if len(h.theta) > 1:
            change = abs(h.theta[-1] - h.theta[-2]) / abs(h.theta[-2])
            self._calm = self._calm + 1 if change < self.rtol else 0
            h.converged = self._calm >= self.patience
        if not h.converged:
            self.rho = self.compliance.solver.oc_update(self.rho, g, self.volume, self.move,
                                                        self.eta, self.rho_min)
        return h.theta[-1]

    def run(self, max_cycles: int) -> DesignHistory:
        for _ in range(max_cycles):
            self.step()
            if self.history.converged:
                break
        return self.history

    def close(self):
        self.compliance.close()
