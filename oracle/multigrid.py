"""Space-time multigrid components (Sections 3-6) written out literally.

* Coarsening strategies: Algorithm 2 (uniform lambda), Algorithm 3 (effective
  anisotropy lambda_eff = sqrt(min lambda_e * max lambda_e), Section 4) and the
  small-feature guard of Algorithm 4 (Section 6).
* Rediscretisation (Section 5.1): interpolation C (causal) or B (bilinear in time),
  reassembly K (average k), D (average chi), R (average resistivity 1/k) or P
  (Galerkin projection R J P, for which lambda_eff uses K-averaged proxies).
* Transfers: prolongation P from the stencils of Section 3.1 / 5.1 and restriction
  R = s P^T with s = 1 for x- and s = 1/2 for t- and full coarsening.
* Damped pointwise Jacobi smoother with omega = 1/2 (Section 3.1).
* Algorithm 1 (V-cycle), zero initial guess, relative residual, termination rule and
  convergence-factor estimate (Section 3.1).

Readings of points the paper leaves open (each stated once here):
* Number of levels: ``max_levels`` when given (the paper's experiments fix N_l);
  otherwise keep coarsening while the current level has more than
  ``min_coarse_dofs`` DOFs.  If the chosen direction cannot halve the grid the other
  direction is taken; if neither can, coarsening stops.
* Ties lambda_eff == lambda_crit choose x-coarsening (Algorithm 3 uses a strict <).
* The coarsest level is solved exactly by time stepping (``direct_solve``).
* The restricted residual is not masked at Dirichlet DOFs (Appendix A: restriction
  mixes interior and Dirichlet residuals).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .discretisation import (Level, Material, apply_J, diag_J, direct_solve, dofs, simp)

__all__ = [
    "Options", "Hierarchy", "lambda_eff", "d_eff_simp", "coarsen", "build_hierarchy",
    "prolongation_1d", "transfer_pair", "prolong", "restrict", "jacobi",
    "vcycle", "SolveResult", "stmg_solve", "galerkin_level",
]


@dataclass
class Options:
    """STMG settings.  Defaults: nu = 2, omega = 1/2, lambda_crit = 0.25, C + R."""
    nu: int = 2
    omega: float = 0.5
    lambda_crit: float = 0.25
    max_levels: int = 0              # 0: stop by min_coarse_dofs instead
    min_coarse_dofs: int = 1024
    M_min_elems: int = 0             # Algorithm 4 guard (0 disables)
    interp: str = "C"                # 'C' causal, 'B' bilinear in time
    reassembly: str = "R"            # 'K', 'D', 'R', 'P'
    deff_mode: str = "field"         # 'field' (Algorithm 3) or 'simp' (Section 7.2)
    material: Material | None = None  # needed for 'D' and deff_mode 'simp'
    force_path: str | None = None    # e.g. "xxt": fixed coarsening directions
    tol: float = 1e-10
    diverge: float = 1e9
    max_cycles: int = 100


# --------------------------------------------------------------------------------------
# Coarsening decision (Algorithms 2-4)
# --------------------------------------------------------------------------------------

def lambda_eff(level: Level) -> float:
    """lambda_eff = D_eff dt / dx^2 with D_eff = sqrt(min_e D_e max_e D_e), D_e = k_e / c_e
    (Section 4, eq. lambda eff def 1).  For uniform material it reduces to the lambda
    of Algorithm 2."""
    d = level.k / level.c
    return float(np.sqrt(np.min(d) * np.max(d)) * level.tau / level.h ** 2)


def d_eff_simp(material: Material) -> float:
    """Field-independent D_eff of Section 7.2: sqrt(D_SIMP(0) D_SIMP(1)), using the
    extrema stated there (eq. D_SIMP extrema)."""
    d0 = material.k_ins / material.c_ins
    d1 = material.k_con / material.c_con
    return float(np.sqrt(d0 * d1))


def coarsen(level: Level, direction: str, opts: Options) -> Level:
    """Next coarser level by x- or t-semi-coarsening (Section 3.1) with the
    coefficient rule of the chosen reassembly method (Section 5.1)."""
    if direction == "f":          # full space-time coarsening (Section 3.1)
        return coarsen(coarsen(level, "t", opts), "x", opts)
    if direction == "t":
        if level.n_t % 2 or level.n_t < 2:
            raise ValueError("cannot t-coarsen")
        return Level(level.n_el, level.n_t // 2, level.h, 2.0 * level.tau,
                     level.k.copy(), level.c.copy(),
                     None if level.chi is None else level.chi.copy())
    if direction != "x":
        raise ValueError(direction)
    if level.n_el % 2 or level.n_el < 2:
        raise ValueError("cannot x-coarsen")
    ka, kb = level.k[0::2], level.k[1::2]
    ca, cb = level.c[0::2], level.c[1::2]
    chi = None
    if opts.reassembly in ("K", "P"):          # eq. K method def (P uses it as a proxy)
        k = (ka + kb) / 2.0
        c = (ca + cb) / 2.0
    elif opts.reassembly == "R":               # resistivity averaging
        rho = (1.0 / ka + 1.0 / kb) / 2.0
        k = 1.0 / rho
        c = (ca + cb) / 2.0
    elif opts.reassembly == "D":               # design-field averaging, then SIMP
        m = opts.material
        chi = (level.chi[0::2] + level.chi[1::2]) / 2.0
        k = simp(chi, m.k_ins, m.k_con, m.p_k)
        c = simp(chi, m.c_ins, m.c_con, m.p_c)
    else:
        raise ValueError(opts.reassembly)
    if chi is None and level.chi is not None:
        chi = (level.chi[0::2] + level.chi[1::2]) / 2.0
    return Level(level.n_el // 2, level.n_t, 2.0 * level.h, level.tau, k, c, chi)


@dataclass
class Hierarchy:
    levels: list
    directions: list      # directions[l] builds levels[l+1] from levels[l]
    lambdas: list         # lambda_eff evaluated on each non-coarsest level
    opts: Options
    galerkin: list = field(default_factory=list)   # sparse J per level for 'P'

    @property
    def path(self) -> str:
        return "".join(self.directions)


def build_hierarchy(fine: Level, opts: Options) -> Hierarchy:
    """Algorithm 3 (Algorithm 4 when opts.M_min_elems > 0) from level 1."""
    levels, dirs, lams = [fine], [], []
    while True:
        cur = levels[-1]
        if opts.force_path is not None:
            if len(dirs) == len(opts.force_path):
                break
        elif opts.max_levels:
            if len(levels) == opts.max_levels:
                break
        elif dofs(cur) <= opts.min_coarse_dofs:
            break
        if opts.deff_mode == "simp":
            lam = d_eff_simp(opts.material) * cur.tau / cur.h ** 2
        else:
            lam = lambda_eff(cur)
        want = "t" if lam < opts.lambda_crit else "x"
        if opts.M_min_elems and cur.n_el / 2 < opts.M_min_elems:
            want = "t"
        if opts.force_path is not None:
            want = opts.force_path[len(dirs)]
        can = {"x": cur.n_el % 2 == 0 and cur.n_el >= 2,
               "t": cur.n_t % 2 == 0 and cur.n_t >= 2}
        can["f"] = can["x"] and can["t"]
        if not can[want]:
            if opts.force_path is not None:
                raise ValueError("forced path cannot be realised")
            want = "t" if want == "x" else "x"
            if not can[want]:
                break
        lams.append(lam)
        dirs.append(want)
        levels.append(coarsen(cur, want, opts))
    h = Hierarchy(levels, dirs, lams, opts)
    if opts.reassembly == "P":
        h.galerkin = _galerkin_operators(h)
    return h


# --------------------------------------------------------------------------------------
# Transfers (Section 3.1 and Section 5.1)
# --------------------------------------------------------------------------------------

def prolongation_1d(n_fine_intervals: int, kind: str) -> sp.csr_matrix:
    """1-D prolongation from n/2 + 1 coarse points to n + 1 fine points.

    kind 'x'  : linear in space, stencil 1/2 ]1 2 1[ : fine 2I <- 1, fine 2I+-1 <- 1/2.
    kind 'tC' : causal in time: coarse level J is copied to fine levels 2J and 2J+1.
    kind 'tB' : linear in time: fine 2J <- 1, fine 2J+-1 <- 1/2.
    Stencils give where a coarse value is distributed to (Section 3.1).
    """
    nf, nc = n_fine_intervals + 1, n_fine_intervals // 2 + 1
    P = sp.lil_matrix((nf, nc))
    for J in range(nc):
        P[2 * J, J] = 1.0
        if kind in ("x", "tB"):
            if 2 * J - 1 >= 0:
                P[2 * J - 1, J] = 0.5
            if 2 * J + 1 < nf:
                P[2 * J + 1, J] = 0.5
        elif kind == "tC":
            if 2 * J + 1 < nf:
                P[2 * J + 1, J] = 1.0
        else:
            raise ValueError(kind)
    return P.tocsr()


def transfer_pair(fine: Level, direction: str, interp: str = "C"):
    """(P_t, P_x, s) such that P z = P_t Z P_x^T on 2-D arrays and R = s P^T.

    For row-major (time-major) flattening this is P = kron(P_t, P_x)."""
    if direction == "x":
        Pt = sp.identity(fine.n_t + 1, format="csr")
        Px = prolongation_1d(fine.n_el, "x")
        s = 1.0
    elif direction == "t":
        Pt = prolongation_1d(fine.n_t, "tC" if interp == "C" else "tB")
        Px = sp.identity(fine.n_el + 1, format="csr")
        s = 0.5
    elif direction == "f":        # full space-time coarsening (Section 3.2 only)
        Pt = prolongation_1d(fine.n_t, "tC" if interp == "C" else "tB")
        Px = prolongation_1d(fine.n_el, "x")
        s = 0.5
    else:
        raise ValueError(direction)
    return Pt, Px, s


def prolong(fine: Level, direction: str, z: np.ndarray, interp: str = "C") -> np.ndarray:
    Pt, Px, _ = transfer_pair(fine, direction, interp)
    return np.asarray(Pt @ (Px @ z.T).T)


def restrict(fine: Level, direction: str, r: np.ndarray, interp: str = "C") -> np.ndarray:
    """R r = s P^T r  (Section 3.1)."""
    Pt, Px, s = transfer_pair(fine, direction, interp)
    return s * np.asarray(Pt.T @ (Px.T @ r.T).T)


# --------------------------------------------------------------------------------------
# Galerkin reassembly (P method)
# --------------------------------------------------------------------------------------

def _sparse_J_by_columns(level: Level, transpose: bool = False) -> sp.csr_matrix:
    """J as a sparse matrix, one application of J per unit vector (tiny grids)."""
    n = dofs(level)
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(sp.csr_matrix(apply_J(level, e.reshape(level.shape), transpose).reshape(-1, 1)))
    return sp.hstack(cols).tocsr()


def _sparse_J(level: Level, transpose: bool = False) -> sp.csr_matrix:
    """J as a sparse matrix from 9 applications of J.  Row (n, i) of J (and of J^T)
    involves only columns (n + dt, i + dx) with |dt|, |dx| <= 1, so the unit vectors
    of all DOFs (m, j) with m = a, j = b (mod 3) have images that do not overlap:
    applying J to their sum gives column (m, j) in the rows (m + dt, j + dx)."""
    nt1, n1 = level.shape
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            e = np.zeros(level.shape)
            e[a::3, b::3] = 1.0
            y = apply_J(level, e, transpose)
            m, j = np.meshgrid(np.arange(a, nt1, 3), np.arange(b, n1, 3), indexing="ij")
            m, j = m.ravel(), j.ravel()
            for dt in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    r, c = m + dt, j + dx
                    ok = (r >= 0) & (r < nt1) & (c >= 0) & (c < n1)
                    v = y[r[ok], c[ok]]
                    nz = v != 0.0
                    rows.append((r[ok] * n1 + c[ok])[nz])
                    cols.append((m[ok] * n1 + j[ok])[nz])
                    vals.append(v[nz])
    n = nt1 * n1
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def _galerkin_operators(h: Hierarchy):
    """J^(l+1) = R^(l) J^(l) P^(l) (Section 5.1, P method); tiny grids only."""
    mats = [_sparse_J(h.levels[0])]
    for l, d in enumerate(h.directions):
        Pt, Px, s = transfer_pair(h.levels[l], d, h.opts.interp)
        P = sp.kron(Pt, Px).tocsr()
        mats.append((s * P.T @ mats[-1] @ P).tocsr())
    return mats


def galerkin_level(h: Hierarchy, l: int):
    return h.galerkin[l]


# --------------------------------------------------------------------------------------
# Smoother and V-cycle (Section 3.1, Algorithm 1)
# --------------------------------------------------------------------------------------

def _apply(h: Hierarchy, l: int, u, transpose):
    if h.galerkin and l > 0:
        A = h.galerkin[l].T if transpose else h.galerkin[l]
        return np.asarray(A @ u.ravel()).reshape(u.shape)
    return apply_J(h.levels[l], u, transpose)


def _diag(h: Hierarchy, l: int):
    if h.galerkin and l > 0:
        return h.galerkin[l].diagonal().reshape(h.levels[l].shape)
    return diag_J(h.levels[l])


def jacobi(h: Hierarchy, l: int, u, b, nu: int, transpose: bool = False):
    """nu steps of u <- u + omega D^-1 (b - J u)  (Section 3.1)."""
    D = _diag(h, l)
    for _ in range(nu):
        u = u + h.opts.omega * (b - _apply(h, l, u, transpose)) / D
    return u


def _coarsest(h: Hierarchy, l: int, b, transpose):
    if h.galerkin and l > 0:
        import scipy.sparse.linalg as spla
        A = h.galerkin[l].T.tocsc() if transpose else h.galerkin[l].tocsc()
        return spla.spsolve(A, b.ravel()).reshape(b.shape)
    return direct_solve(h.levels[l], b, transpose)


def vcycle(h: Hierarchy, l: int, u, b, transpose: bool = False):
    """Algorithm 1.  The adjoint uses (J^(l))^T on every level with the same P and R
    (Section 7.2)."""
    if l == len(h.levels) - 1:
        return _coarsest(h, l, b, transpose)
    nu = h.opts.nu
    u = jacobi(h, l, u, b, nu, transpose)
    d = h.directions[l]
    bc = restrict(h.levels[l], d, b - _apply(h, l, u, transpose), h.opts.interp)
    z = vcycle(h, l + 1, np.zeros(h.levels[l + 1].shape), bc, transpose)
    u = u + prolong(h.levels[l], d, z, h.opts.interp)
    return jacobi(h, l, u, b, nu, transpose)


@dataclass
class SolveResult:
    u: np.ndarray
    status: str                       # 'converged', 'diverged', 'max_cycles'
    cycles: int
    history: list                     # r_0, r_1, ..., r_N
    iterates: list | None = None

    @property
    def conv_factor(self) -> float:
        """(r_N / r_0)^(1/N)  (Section 3.1)."""
        n = self.cycles
        return float((self.history[n] / self.history[0]) ** (1.0 / n)) if n else float("nan")


def stmg_solve(h: Hierarchy, b, u0=None, transpose: bool = False,
               keep_iterates: bool = False) -> SolveResult:
    """Repeated V-cycles from u = 0 (Section 3.1) until r_n < tol, r_n > diverge or
    n = max_cycles (eq. STMG termination criterion; thresholds are options)."""
    o = h.opts
    u = np.zeros(h.levels[0].shape) if u0 is None else np.array(u0, dtype=np.float64)
    nb = np.linalg.norm(b)
    hist = [float(np.linalg.norm(_apply(h, 0, u, transpose) - b) / nb)]
    its = [] if keep_iterates else None
    status = "max_cycles"
    n = 0
    for n in range(1, o.max_cycles + 1):
        u = vcycle(h, 0, u, b, transpose)
        r = float(np.linalg.norm(_apply(h, 0, u, transpose) - b) / nb)
        hist.append(r)
        if keep_iterates:
            its.append(u.copy())
        if not np.isfinite(r) or r > o.diverge:
            status = "diverged"
            break
        if r < o.tol:
            status = "converged"
            break
    return SolveResult(u, status, n, hist, its)
