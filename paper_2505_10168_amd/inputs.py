"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws and shapes input data (design fields, heat loads, request
streams).  It contains none of the solver's arithmetic: no material interpolation,
no discretisation, no multigrid step.  Both the HIP path and the CPU oracle receive
the arrays produced here, so neither depends on the other.

Design fields are element densities rho_e in [0, 1] (one per element).  Heat loads
are element-wise and per time level, shape (n_t + 1, n_el), row 0 unused (the
initial condition carries no load), matching Section 2.2 where q is element-wise
constant and evaluated at the backward-Euler time points t_n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------------------
# Design fields
# --------------------------------------------------------------------------------------

def block_density(n_el: int, block: int, seed: int, p: float = 0.5,
                  first_on: bool = False) -> np.ndarray:
    """Piecewise-constant 0/1 density in blocks of ``block`` elements.

    Each block is 1 with probability ``p``.  A draw with every block equal is redrawn
    (the field is meant to be high contrast), deterministically from the same seed;
    with ``first_on`` a draw whose first block (next to the cold end x = 0) is
    insulating is redrawn too.
    """
    if n_el % block != 0:
        raise ValueError("n_el must be a multiple of the block length")
    rng = np.random.default_rng(seed)
    nb = n_el // block
    while True:
        bits = (rng.random(nb) < p).astype(np.float64)
        if (nb == 1 or bits.min() != bits.max()) and (not first_on or bits[0] == 1.0):
            break
    return np.repeat(bits, block)


def box_filtered_uniform_density(n_el: int, width: int, seed: int) -> np.ndarray:
    """I.i.d. U[0,1) densities smoothed by a centred box filter of ``width`` elements.

    At the ends the window is truncated and the average is taken over the elements
    that are present.
    """
    rng = np.random.default_rng(seed)
    raw = rng.random(n_el)
    half = width // 2
    csum = np.concatenate([[0.0], np.cumsum(raw)])
    lo = np.clip(np.arange(n_el) - half, 0, n_el)
    hi = np.clip(np.arange(n_el) + half + 1, 0, n_el)
    return (csum[hi] - csum[lo]) / (hi - lo)


def uniform_random_density(n_el: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(n_el)


def f01(v):
    """Clamp to [0, 1] (the function f01 of Section 4)."""
    return np.clip(v, 0.0, 1.0)


def element_centres(n_el: int, length: float) -> np.ndarray:
    """x_e = (e + 1/2) dx with dx = L / n_el (Section 2.2)."""
    return (np.arange(n_el) + 0.5) * (length / n_el)


def ramp_design(n_el: int, length: float, alpha: float, x_offset: float) -> np.ndarray:
    """Design field of problems 1-7: chi_e = f01(1/2 - alpha (x_e - x_offset)) (Section 4)."""
    return f01(0.5 - alpha * (element_centres(n_el, length) - x_offset))


def thin_insulator_design(n_el: int, length: float, frac: float) -> np.ndarray:
    """Design field of problem 8: two conductors split by a thin insulator (Section 5.2)."""
    x = element_centres(n_el, length)
    return f01(np.abs((x - length / 2) / length) * 2.0 / frac - 1.0)


def thin_conductor_design(n_el: int, length: float, frac: float) -> np.ndarray:
    """Design field of problem 9: the complement of problem 8 (Section 5.2)."""
    return 1.0 - thin_insulator_design(n_el, length, frac)


# --------------------------------------------------------------------------------------
# Heat loads
# --------------------------------------------------------------------------------------

def paper_heat_load(n_el: int, n_t: int, length: float, t_final: float) -> np.ndarray:
    """Many-frequency test load of Section 3.1 (eq. heat load), shape (n_t+1, n_el).

    q_{e,j} = (1 + cos(200 [(x_e/L - 1/2)^2 + (t_j/t_T - 1/2)^2])) * 1e6, row 0 unused.
    """
    x = element_centres(n_el, length) / length - 0.5
    t = (np.arange(n_t + 1) * (t_final / n_t)) / t_final - 0.5
    q = (1.0 + np.cos(200.0 * (x[None, :] ** 2 + t[:, None] ** 2))) * 1e6
    q[0, :] = 0.0
    return q


def random_heat_load(n_el: int, n_t: int, seed: int) -> np.ndarray:
    q = np.random.default_rng(seed).random((n_t + 1, n_el))
    q[0, :] = 0.0
    return q


def random_nodal(n_el: int, n_t: int, seed: int) -> np.ndarray:
    """Random space-time nodal vector of shape (n_t+1, n_el+1) (e.g. a right-hand side)."""
    return np.random.default_rng(seed).standard_normal((n_t + 1, n_el + 1))


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_el: int
    n_t: int
    kappa_min: float
    rho: np.ndarray
    length: float = 1.0
    t_final: float = 0.1

    @property
    def dofs(self) -> int:
        return (self.n_el + 1) * (self.n_t + 1)


def workload(name: str) -> Workload:
    """The five benchmark workloads (heat source q = 1, L = 1, t_T = 0.1, c = 1)."""
    if name == "uniform_64x64":
        return Workload(name, 64, 64, 1.0, np.ones(64))
    if name == "block_1024x4096":
        return Workload(name, 1024, 4096, 1e-3, block_density(1024, 16, seed=2))
    if name == "boxfilt_8192x65536":
        return Workload(name, 8192, 65536, 1e-4, box_filtered_uniform_density(8192, 9, seed=3))
    if name == "block_2048x8192":
        # the gradient workload: its first block conducts, so the rod is thermally
        # connected to the cold end and the design sensitivities are measurable
        return Workload(name, 2048, 8192, 1e-3, block_density(2048, 16, seed=4, first_on=True))
    raise KeyError(name)


# --------------------------------------------------------------------------------------
# Serving request stream
# --------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n_el: int
    n_t: int
    kappa_min: float
    rho: np.ndarray
    with_adjoint: bool

    @property
    def dofs(self) -> int:
        return (self.n_el + 1) * (self.n_t + 1)


def log_uniform_size(rng, lo: int, hi: int) -> int:
    """exp(U(ln lo, ln hi)) rounded to two significant bits, i.e. to one of
    {4, 5, 6, 7} * 2^q (four sizes per octave, each halving q times), kept in [lo, hi]."""
    v = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    q = max(int(math.floor(math.log2(v))) - 2, 0)
    return int(min(max(round(v / 2 ** q) * 2 ** q, lo), hi))


def request_stream(n: int, rate_per_s: float, seed: int = 5,
                   el_range=(128, 4096), t_range=(256, 16384)) -> list[Request]:
    """Poisson arrivals of solve requests with log-uniform grid sizes.

    Elements log-uniform in el_range and time steps log-uniform in t_range, each
    rounded to two significant bits ({4, 5, 6, 7} * 2^q: sizes that halve q times, so
    that the hierarchy can coarsen far in both directions; el_range starts at 64 or
    more, so fields are whole blocks of 16); block-16 0/1 density fields, kappa_min from
    {1e-2, 1e-3, 1e-4}; exactly half of the requests also ask for the adjoint and
    gradient, in shuffled order.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n) if rate_per_s > 0 else np.zeros(n)
    arrivals = np.cumsum(gaps)
    adj = np.array([True] * (n // 2) + [False] * (n - n // 2))
    rng.shuffle(adj)
    out = []
    for r in range(n):
        n_el = log_uniform_size(rng, el_range[0], el_range[1])
        n_t = log_uniform_size(rng, t_range[0], t_range[1])
        kmin = float(rng.choice([1e-2, 1e-3, 1e-4]))
        rho = block_density(n_el, 16, seed=int(rng.integers(0, 2**31)))
        out.append(Request(r, float(arrivals[r]), n_el, n_t, kmin, rho, bool(adj[r])))
    return out


def log2_int(v: int) -> int:
    return int(round(math.log2(v)))
