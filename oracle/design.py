"""Design update of the Section 7 optimisation problem, written out plainly.

Test infrastructure only (see the package docstring).

Section 7.1 minimises Theta over the design field subject to the box constraint
0 <= chi <= 1 and the volume constraint (integral of chi over the rod) <= L/2, i.e.
mean(chi) <= 1/2 on the uniform mesh.  The paper updates the design with MMA, which
it only cites; the update here is the classical optimality-criteria (OC) step for a
single volume constraint (Bendsoe, "Optimization of Structural Topology, Shape, and
Material", 1995, Section 1.2):

    D_e       = max(-g_e, 0)
    lo_e      = max(chi_min, chi_e - m),   hi_e = min(1, chi_e + m)
    x_e(lam)  = chi_e (D_e / lam)^eta
    chi_e'    = min(max(x_e(lam), lo_e), hi_e)

with the multiplier lam > 0 chosen so that mean(chi') meets the volume bound.
mean(chi'(lam)) does not increase with lam, so lam is found by bisection on log(lam)
over [1e-40, 1e40] * max D (mid = sqrt(a) sqrt(b), 96 halvings): a step goes up when
the trial volume exceeds the bound.  When even the smallest lam leaves the volume
below the bound the constraint is inactive and every element with D_e > 0 goes to hi_e.

The design loop evaluates Theta and g by direct solves (the exact solutions the STMG
solves converge to) and stops by the rule of Section 7.2: the relative change of
Theta stays below 0.1 % for 5 consecutive cycles.
"""
from __future__ import annotations

import math

import numpy as np

from .discretisation import Material, direct_solve, load_vector, make_fine_level
from .sensitivity import adjoint_rhs, gradient, objective

__all__ = ["oc_update", "oc_multiplier", "theta_and_gradient", "design_loop"]

OC_BRACKET = 1e40
OC_HALVINGS = 96


def _oc_trial(chi, drive, lam, lo, hi, eta):
    return np.minimum(np.maximum(chi * (drive / lam) ** eta, lo), hi)


def oc_multiplier(chi, grad, volume: float, move: float = 0.2, eta: float = 0.5,
                  chi_min: float = 1e-3) -> float:
    """The multiplier lam of the OC step (bisection on log lam, see the module text)."""
    chi = np.asarray(chi, dtype=np.float64)
    drive = np.maximum(-np.asarray(grad, dtype=np.float64), 0.0)
    lo = np.maximum(chi_min, chi - move)
    hi = np.minimum(1.0, chi + move)
    scale = float(drive.max()) if float(drive.max()) > 0.0 else 1.0
    a, b = scale / OC_BRACKET, scale * OC_BRACKET
    for _ in range(OC_HALVINGS):
        mid = math.sqrt(a) * math.sqrt(b)
        if _oc_trial(chi, drive, mid, lo, hi, eta).sum() / chi.size > volume:
            a = mid
        else:
            b = mid
    return math.sqrt(a) * math.sqrt(b)


def oc_update(chi, grad, volume: float, move: float = 0.2, eta: float = 0.5,
              chi_min: float = 1e-3) -> np.ndarray:
    """The new design chi' of the OC step."""
    chi = np.asarray(chi, dtype=np.float64)
    drive = np.maximum(-np.asarray(grad, dtype=np.float64), 0.0)
    lo = np.maximum(chi_min, chi - move)
    hi = np.minimum(1.0, chi + move)
    lam = oc_multiplier(chi, grad, volume, move, eta, chi_min)
    return _oc_trial(chi, drive, lam, lo, hi, eta)


def theta_and_gradient(chi, material: Material, n_t: int, length: float, t_final: float,
                       q, theta_ref: float):
    """Theta (Section 7.1) and dTheta/dchi (Section 7.2) from direct solves."""
    lv = make_fine_level(chi, material, n_t, length, t_final)
    b = load_vector(lv, q)
    u = direct_solve(lv, b)
    lam = direct_solve(lv, adjoint_rhs(lv, b, theta_ref), transpose=True)
    return objective(lv, b, u, theta_ref), gradient(lv, material, chi, u, lam)


def design_loop(chi0, material: Material, n_t: int, length: float, t_final: float, q,
                theta_ref: float, volume: float, max_cycles: int, move: float = 0.2,
                eta: float = 0.5, chi_min: float = 1e-3, rtol: float = 1e-3,
                patience: int = 5):
    """OC design loop; returns (designs, thetas): designs[k] is the design of cycle k
    and thetas[k] its Theta.  Stops after `patience` consecutive cycles whose relative
    change of Theta is below rtol (Section 7.2), or after max_cycles."""
    chi = np.asarray(chi0, dtype=np.float64).copy()
    designs, thetas = [], []
    calm = 0
    for _ in range(max_cycles):
        th, g = theta_and_gradient(chi, material, n_t, length, t_final, q, theta_ref)
        designs.append(chi.copy())
        thetas.append(th)
        if len(thetas) > 1:
            calm = calm + 1 if abs(thetas[-1] - thetas[-2]) < rtol * abs(thetas[-2]) else 0
            if calm >= patience:
                break
        chi = oc_update(chi, g, volume, move, eta, chi_min)
    return designs, thetas
