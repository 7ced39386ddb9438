"""Objective, adjoint and sensitivities (Section 7), written out literally.

Theta = b^T u dt / Theta_ref (Section 7.1) and the discrete adjoint
J^T Lambda = b dt / Theta_ref (Section 7.2).  The paper names the discrete adjoint
method but does not print the sensitivity formula; it follows from differentiating
Theta(rho) = (dt/Theta_ref) b^T J(rho)^{-1} b with b independent of the design:

    dTheta/drho_e = - Lambda^T (dJ/drho_e) u.

With J = B J_Neu B + W (I - B) (Appendix A) the W term is multiplied by the
Dirichlet entries u_D = b_D / W = 0 of the exact solution, so only B J_Neu B
contributes.  J_Neu depends on rho_e through element e's stiffness
(k'_e / h) [[1, -1], [-1, 1]] on every diagonal block and its capacity
(c'_e h / 6) [[2, 1], [1, 2]] on the diagonal (+1/dt) and sub-diagonal (-1/dt)
blocks.  Writing u~ = B u and Lambda~ = B Lambda:

    g_e = - sum_{n=1}^{N_t} [ (k'_e / h) (L_{e+1,n} - L_{e,n}) (u_{e+1,n} - u_{e,n})
                             + (c'_e h / (6 dt)) (L_{e,n}, L_{e+1,n}) [[2,1],[1,2]]
                               (du_{e,n}, du_{e+1,n})^T ],   du_n = u_n - u_{n-1}

with all u, L taken from u~, Lambda~ and k'_e, c'_e the SIMP derivatives.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .discretisation import Level, Material, dirichlet_mask, simp_derivative

__all__ = ["objective", "adjoint_rhs", "gradient"]


def objective(level: Level, b: np.ndarray, u: np.ndarray, theta_ref: float = 1.0) -> float:
    """Theta = b^T u dt / Theta_ref  (Section 7.1)."""
    return float(np.sum(b * u) * level.tau / theta_ref)


def adjoint_rhs(level: Level, b: np.ndarray, theta_ref: float = 1.0) -> np.ndarray:
    """(dTheta/du)^T = b dt / Theta_ref  (Section 7.2)."""
    return b * (level.tau / theta_ref)


def gradient(level: Level, material: Material, chi: np.ndarray, u: np.ndarray,
             lam: np.ndarray) -> np.ndarray:
    """dTheta/dchi_e by the discrete adjoint method (see the module docstring)."""
    B = dirichlet_mask(level)
    ut, lt = B * u, B * lam
    kp = simp_derivative(chi, material.k_ins, material.k_con, material.p_k)
    cp = simp_derivative(chi, material.c_ins, material.c_con, material.p_c)
    h, tau = level.h, level.tau
    du_x = ut[1:, 1:] - ut[1:, :-1]          # u_{e+1,n} - u_{e,n}, n = 1..N_t
    dl_x = lt[1:, 1:] - lt[1:, :-1]
    g = -(kp / h) * np.sum(dl_x * du_x, axis=0)
    dut = ut[1:] - ut[:-1]                    # u_n - u_{n-1}, n = 1..N_t
    la, lb = lt[1:, :-1], lt[1:, 1:]
    da, db = dut[:, :-1], dut[:, 1:]
    mass = la * (2 * da + db) + lb * (da + 2 * db)
    g -= (cp * h / (6.0 * tau)) * np.sum(mass, axis=0)
    return g
