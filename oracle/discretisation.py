"""Discretisation of the 1D transient heat equation (Section 2) and its boundary
treatment (Appendix A), written out literally in NumPy float64.

Conventions
-----------
A space-time nodal vector is a 2-D array ``u[n, i]`` of shape (N_t+1, N_el+1): time
level n = 0..N_t (rows, stacked T_0, T_1, ... as in the all-at-once system of
Section 2.2) and node i = 0..N_el (columns).  Node 0 is x = 0 (Dirichlet, T = 0),
node N_el is x = L (adiabatic).  Time level 0 is the initial condition, which
Appendix A also treats as a Dirichlet condition.

Element coefficients k_e, c_e are element-wise constant (Section 2.2).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np
from scipy.linalg import solve_banded

__all__ = [
    "Material", "Level", "simp", "simp_derivative", "make_fine_level",
    "mass_matrix_diagonals", "stiffness_matrix_diagonals", "w_diri",
    "tridiag_apply", "stiffness_apply", "dirichlet_mask", "apply_J", "diag_J", "load_vector",
    "dense_J", "direct_solve", "relative_residual", "dofs",
]


# --------------------------------------------------------------------------------------
# Materials (Section 2.1)
# --------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Material:
    """Two-material SIMP parametrisation (Section 2.1, eqs. SIMP k and SIMP c).

    The paper uses p_k = 3 and p_c = 2.  A constant heat capacity is obtained with
    c_ins == c_con.
    """
    k_ins: float
    k_con: float
    c_ins: float
    c_con: float
    p_k: float = 3.0
    p_c: float = 2.0


def simp(chi, v_ins: float, v_con: float, p: float):
    """v(chi) = v_ins + (v_con - v_ins) chi^p  (Section 2.1, eqs. SIMP k / SIMP c)."""
    chi = np.asarray(chi, dtype=np.float64)
    return v_ins + (v_con - v_ins) * chi ** p


def simp_derivative(chi, v_ins: float, v_con: float, p: float):
    """d v / d chi = p (v_con - v_ins) chi^(p-1)."""
    chi = np.asarray(chi, dtype=np.float64)
    if p == 0:
        return np.zeros_like(chi)
    return p * (v_con - v_ins) * chi ** (p - 1.0)


# --------------------------------------------------------------------------------------
# Levels
# --------------------------------------------------------------------------------------

@dataclass
class Level:
    """One uniform space-time grid with element coefficients.

    n_el elements of width h, n_t backward-Euler steps of length tau (Section 2.2).
    ``chi`` is kept only for the D reassembly method (Section 5.1).
    """
    n_el: int
    n_t: int
    h: float
    tau: float
    k: np.ndarray
    c: np.ndarray
    chi: np.ndarray | None = None
    w_override: float | None = None
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.n_t + 1, self.n_el + 1)

    @property
    def W(self) -> float:
        return w_diri(self) if self.w_override is None else self.w_override

    def copy(self, **kw):
        return replace(self, **kw)


def dofs(level: Level) -> int:
    return (level.n_el + 1) * (level.n_t + 1)


def make_fine_level(chi, material: Material, n_t: int, length: float, t_final: float,
                    w_override: float | None = None) -> Level:
    """Level 1 from the design field: dx = L/N_el, dt = t_T/N_t (Section 2.2) and
    k_e = k_SIMP(chi_e), c_e = c_SIMP(chi_e) (Section 2.1)."""
    chi = np.asarray(chi, dtype=np.float64)
    n_el = chi.size
    k = simp(chi, material.k_ins, material.k_con, material.p_k)
    c = simp(chi, material.c_ins, material.c_con, material.p_c)
    return Level(n_el, n_t, length / n_el, t_final / n_t, k, c, chi.copy(), w_override)


# --------------------------------------------------------------------------------------
# Spatial matrices (Section 2.2: linear shape functions, element-wise constant k, c)
# --------------------------------------------------------------------------------------

def mass_matrix_diagonals(level: Level):
    """Heat-capacity matrix C assembled with only natural boundary conditions.

    Element e (nodes e, e+1) contributes c_e h / 6 * [[2, 1], [1, 2]].
    Returns (main diagonal of length N+1, off diagonal of length N); C is symmetric.
    """
    n, h, c = level.n_el, level.h, level.c
    main = np.zeros(n + 1)
    main[:-1] += 2.0 * c * h / 6.0
    main[1:] += 2.0 * c * h / 6.0
    off = c * h / 6.0
    return main, off


def stiffness_matrix_diagonals(level: Level):
    """Conductivity matrix K: element e contributes k_e / h * [[1, -1], [-1, 1]]."""
    n, h, k = level.n_el, level.h, level.k
    main = np.zeros(n + 1)
    main[:-1] += k / h
    main[1:] += k / h
    off = -k / h
    return main, off


def w_diri(level: Level) -> float:
    """W_Diri^(l) = max_e c_e dx/dt + max_e k_e / dx  (Appendix A)."""
    return float(np.max(level.c) * level.h / level.tau + np.max(level.k) / level.h)


def tridiag_apply(main, off, x):
    """y = T x along the last axis for the symmetric tridiagonal T(main, off)."""
    y = main * x
    y[..., :-1] += off * x[..., 1:]
    y[..., 1:] += off * x[..., :-1]
    return y


def dirichlet_mask(level: Level) -> np.ndarray:
    """Diagonal of B (Appendix A): 0 at Dirichlet DOFs (node 0 and time level 0), else 1."""
    b = np.ones(level.shape)
    b[0, :] = 0.0
    b[:, 0] = 0.0
    return b


def stiffness_apply(level: Level, x: np.ndarray) -> np.ndarray:
    """K x assembled element by element: element e adds the flux (k_e / h)(x_e - x_{e+1})
    to node e and subtracts it from node e+1 (linear elements, Section 2.2)."""
    flux = (level.k / level.h) * (x[..., :-1] - x[..., 1:])
    y = np.zeros_like(x)
    y[..., :-1] += flux
    y[..., 1:] -= flux
    return y


def apply_J(level: Level, u: np.ndarray, transpose: bool = False) -> np.ndarray:
    """y = J u (or J^T u) for J = B J_Neu B + W_Diri (I - B)  (Appendix A).

    J_Neu is the all-at-once BE-FE matrix of Section 2.2: time level n >= 1 carries the
    backward-Euler step C (T_n - T_{n-1}) / dt + K T_n; its block row 0 is irrelevant
    since B removes it.  J_Neu^T carries C (T_n - T_{n+1}) / dt + K T_n, with no
    T_{n+1} on the last level.  The step is evaluated in this difference form, as the
    paper writes it, with K applied element by element.
    """
    mm, mo = mass_matrix_diagonals(level)
    tau = level.tau
    B = dirichlet_mask(level)
    ub = B * u
    y = np.zeros(level.shape)
    if not transpose:
        d = ub[1:] - ub[:-1]
        y[1:] = tridiag_apply(mm / tau, mo / tau, d) + stiffness_apply(level, ub[1:])
    else:
        d = ub.copy()
        d[:-1] -= ub[1:]
        y[:] = tridiag_apply(mm / tau, mo / tau, d) + stiffness_apply(level, ub)
    return B * y + level.W * (1.0 - B) * u


def diag_J(level: Level) -> np.ndarray:
    """Main diagonal of J (identical for J^T): C_ii/dt + K_ii inside, W_Diri at Dirichlet DOFs."""
    mm, _ = mass_matrix_diagonals(level)
    km, _ = stiffness_matrix_diagonals(level)
    B = dirichlet_mask(level)
    d = np.broadcast_to(mm / level.tau + km, level.shape)
    return B * d + level.W * (1.0 - B)


def load_vector(level: Level, q) -> np.ndarray:
    """b = B b_Neu with b_Neu,n = integral of q(t_n) times the hat functions (Section 2.2).

    ``q`` is either a scalar (uniform heat source) or an element-wise array of shape
    (N_t+1, N_el) with row n the load at t_n (row 0 unused).  With element-wise
    constant q the integral over element e of q_e phi_i is q_e h / 2 for both of its
    nodes.
    """
    n, h = level.n_el, level.h
    if np.isscalar(q):
        q = np.full((level.n_t + 1, n), float(q))
    q = np.asarray(q, dtype=np.float64)
    if q.shape != (level.n_t + 1, n):
        raise ValueError("heat load must have shape (n_t+1, n_el)")
    b = np.zeros(level.shape)
    b[:, :-1] += q * h / 2.0
    b[:, 1:] += q * h / 2.0
    return dirichlet_mask(level) * b


def dense_J(level: Level, transpose: bool = False) -> np.ndarray:
    """Dense all-at-once matrix for tiny grids, assembled block by block from the
    displayed matrix of Section 2.2 and then corrected as in Appendix A."""
    nx, nt = level.n_el + 1, level.n_t + 1
    mm, mo = mass_matrix_diagonals(level)
    km, ko = stiffness_matrix_diagonals(level)
    C = np.diag(mm) + np.diag(mo, 1) + np.diag(mo, -1)
    K = np.diag(km) + np.diag(ko, 1) + np.diag(ko, -1)
    Jn = np.zeros((nt * nx, nt * nx))
    for n in range(1, nt):
        r = slice(n * nx, (n + 1) * nx)
        Jn[r, r] = C / level.tau + K
        Jn[r, (n - 1) * nx:n * nx] = -C / level.tau
    Bd = np.diag(dirichlet_mask(level).ravel())
    J = Bd @ Jn @ Bd + level.W * (np.eye(nt * nx) - Bd)
    return J.T.copy() if transpose else J


# --------------------------------------------------------------------------------------
# Direct solve
# --------------------------------------------------------------------------------------

def direct_solve(level: Level, b: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Exact solution of J u = b (or J^T u = b).

    J is block lower bidiagonal in time once Appendix A has removed the Dirichlet
    rows and columns, so the solve is backward-Euler time stepping: Dirichlet DOFs
    take u = b / W_Diri, and for time levels n = 1..N_t the free nodes solve the
    tridiagonal system (C/dt + K) T_n = b_n + C/dt T_{n-1} (no coupling to level 0).
    The transposed system steps backwards from n = N_t with coupling to n + 1.
    Each tridiagonal solve uses LAPACK's banded solver.
    """
    mm, mo = mass_matrix_diagonals(level)
    km, ko = stiffness_matrix_diagonals(level)
    tau, W = level.tau, level.W
    u = np.zeros(level.shape)
    u[0, :] = b[0, :] / W
    u[:, 0] = b[:, 0] / W
    if level.n_el == 0 or level.n_t == 0:
        return u
    a_main = (mm / tau + km)[1:]
    a_off = (mo / tau + ko)[1:]
    ab = np.zeros((3, level.n_el))
    ab[0, 1:] = a_off
    ab[1, :] = a_main
    ab[2, :-1] = a_off
    m_main, m_off = (mm / tau)[1:], (mo / tau)[1:]
    steps = range(1, level.n_t + 1) if not transpose else range(level.n_t, 0, -1)
    for n in steps:
        rhs = b[n, 1:].copy()
        prev = n - 1 if not transpose else n + 1
        if 1 <= prev <= level.n_t:
            rhs += tridiag_apply(m_main, m_off, u[prev, 1:])
        u[n, 1:] = solve_banded((1, 1), ab, rhs)
    return u


def relative_residual(level: Level, u, b, transpose: bool = False) -> float:
    """r = ||J u - b||_2 / ||b||_2  (Section 3.1)."""
    return float(np.linalg.norm(apply_J(level, u, transpose) - b) / np.linalg.norm(b))
