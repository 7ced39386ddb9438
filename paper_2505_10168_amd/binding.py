"""Thin ctypes binding of libstmg (include/stmg.h).

Argument marshalling only: every step of the solver runs in the HIP library.  Device
memory and streams come from PyTorch (``torch.cuda``); vectors are passed as raw
device pointers of contiguous float64 CUDA tensors.  The functions keep the C names.
If the shared library is missing the import of this module fails loudly: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

# STMG_LIBRARY may point to another build of the library (e.g. a tuning variant).
LIB_PATH = Path(os.environ.get("STMG_LIBRARY") or
                Path(__file__).resolve().parent / "_lib" / "libstmg.so")

STMG_OK, STMG_NOT_CONVERGED, STMG_DIVERGED = 0, 1, 2
STMG_EINVAL, STMG_ENOMEM, STMG_EHIP, STMG_EUNSUPPORTED = -1, -2, -3, -4
STMG_REASSEMBLE_R, STMG_REASSEMBLE_K, STMG_REASSEMBLE_D, STMG_REASSEMBLE_P = 0, 1, 2, 3
STMG_INTERP_C, STMG_INTERP_B = 0, 1
STMG_FP64, STMG_MIXED = 0, 1
STMG_FIELD_DENSITY, STMG_FIELD_CONDUCTIVITY = 0, 1
STMG_MAX_HISTORY = 1024


class stmg_problem(C.Structure):
    _fields_ = [("n_el", C.c_int32), ("n_t", C.c_int32), ("length", C.c_double),
                ("t_final", C.c_double), ("k_ins", C.c_double), ("k_con", C.c_double),
                ("c_ins", C.c_double), ("c_con", C.c_double), ("p_k", C.c_double),
                ("p_c", C.c_double), ("theta_ref", C.c_double), ("q_uniform", C.c_double),
                ("field_kind", C.c_int32)]


class stmg_options(C.Structure):
    _fields_ = [("nu", C.c_int32), ("omega", C.c_double), ("lambda_crit", C.c_double),
                ("max_levels", C.c_int32), ("min_coarse_dofs", C.c_int64),
                ("M_min_elems", C.c_int32), ("reassembly", C.c_int32), ("deff_mode", C.c_int32),
                ("tol", C.c_double), ("diverge", C.c_double), ("max_cycles", C.c_int32),
                ("precision", C.c_int32), ("w_diri_override", C.c_double), ("fused", C.c_int32),
                ("time_kernels", C.c_int32), ("interp", C.c_int32), ("debug_poison", C.c_int32),
                ("inner_cycles", C.c_int32), ("time_levels", C.c_int32)]


class stmg_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("n_levels", C.c_int32),
                ("rel_residual", C.c_double), ("conv_factor", C.c_double),
                ("solve_ms", C.c_double), ("dof_updates", C.c_double),
                ("fine_kernel_ms", C.c_double), ("fine_kernel_bytes", C.c_double),
                ("fine_kernel_launches", C.c_int64), ("fine_passes", C.c_int64),
                ("setup_ms", C.c_double),
                ("path", C.c_char * 128), ("level_cycles", C.c_int32),
                ("level_ms", C.c_double * 64),
                ("history", C.c_double * (STMG_MAX_HISTORY + 1))]


class stmg_info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_el", C.c_int32 * 64), ("n_t", C.c_int32 * 64),
                ("h", C.c_double * 64), ("tau", C.c_double * 64), ("w_diri", C.c_double * 64),
                ("lambda_eff", C.c_double * 64), ("path", C.c_char * 64),
                ("device_bytes", C.c_size_t), ("tail_level", C.c_int32)]


def _load():
    if not LIB_PATH.exists():
        raise ImportError(f"libstmg.so not built ({LIB_PATH}); run __graft_entry__.build()")
    # PyTorch ships its own HIP and HSA runtimes (same SONAME, different file name).
    # Import it first so that libstmg binds to the runtime torch uses: loading the
    # system runtime first would put two HIP runtimes into the process.
    import torch  # noqa: F401
    lib = C.CDLL(str(LIB_PATH))
    P, I, D, VP = C.POINTER, C.c_int, C.c_double, C.c_void_p
    sig = {
        "stmg_default_options": (I, [P(stmg_options)]),
        "stmg_footprint": (I, [P(stmg_problem), P(stmg_options), I, P(C.c_size_t)]),
        "stmg_create": (I, [P(VP), P(stmg_problem), P(stmg_options), VP, VP, VP]),
        "stmg_set_field": (I, [VP, VP]),
        "stmg_set_design": (I, [VP, VP]),
        "stmg_solve_forward": (I, [VP, VP, VP, VP, P(stmg_stats)]),
        "stmg_solve_adjoint": (I, [VP, VP, VP, VP, P(stmg_stats)]),
        "stmg_objective": (I, [VP, VP, P(D)]),
        "stmg_gradient": (I, [VP, VP, VP, VP]),
        "stmg_gradient_noalloc": (I, [P(stmg_problem), VP, VP, VP, VP, VP]),
        "stmg_oc_update": (I, [VP, VP, VP, D, D, D, D, VP]),
        "stmg_get_info": (I, [VP, P(stmg_info)]),
        "stmg_destroy": (I, [VP]),
        "stmg_level_apply": (I, [VP, I, I, VP, VP]),
        "stmg_level_smooth": (I, [VP, I, I, I, VP, VP]),
        "stmg_level_presmooth_restrict": (I, [VP, I, I, I, VP, VP, VP]),
        "stmg_level_prolong_postsmooth": (I, [VP, I, I, I, VP, VP, VP]),
        "stmg_level_coarsest_solve": (I, [VP, I, VP, VP]),
        "stmg_vcycle": (I, [VP, I, VP, VP, P(D)]),
        "stmg_pass_geometry": (I, [I, I, I, I, I, P(I), P(I), P(I), P(I)]),
        "stmg_stream_calibrate": (I, [VP, VP, D, VP, C.c_int64, I, VP]),
        "stmg_status_string": (C.c_char_p, [I]),
        "stmg_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# Every symbol declared in include/stmg.h, for the export test.
EXPORTED = [
    "stmg_default_options", "stmg_footprint", "stmg_create", "stmg_set_field", "stmg_set_design",
    "stmg_solve_forward", "stmg_solve_adjoint", "stmg_objective", "stmg_gradient",
    "stmg_gradient_noalloc", "stmg_oc_update",
    "stmg_get_info", "stmg_destroy", "stmg_level_apply", "stmg_level_smooth",
    "stmg_level_presmooth_restrict", "stmg_level_prolong_postsmooth",
    "stmg_level_coarsest_solve", "stmg_vcycle", "stmg_pass_geometry", "stmg_stream_calibrate",
    "stmg_status_string",
    "stmg_last_error",
]


class StmgError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.stmg_last_error().decode() or lib.stmg_status_string(code).decode()
        super().__init__(f"{where}: {lib.stmg_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code: int, where: str) -> int:
    if code < 0:
        raise StmgError(code, where)
    return code


def _ptr(t) -> int | None:
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not (t.is_cuda and t.dtype.is_floating_point and t.dtype.itemsize == 8 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---- functions with the C names ------------------------------------------------------

def stmg_default_options() -> stmg_options:
    o = stmg_options()
    _check(lib.stmg_default_options(C.byref(o)), "stmg_default_options")
    return o


def stmg_footprint(problem: stmg_problem, options: stmg_options, with_adjoint: bool = False) -> int:
    out = C.c_size_t()
    _check(lib.stmg_footprint(C.byref(problem), C.byref(options), int(bool(with_adjoint)),
                              C.byref(out)), "stmg_footprint")
    return out.value


def stmg_create(problem: stmg_problem, options: stmg_options, rho, q=None, stream=None) -> int:
    h = C.c_void_p()
    _check(lib.stmg_create(C.byref(h), C.byref(problem), C.byref(options), _ptr(rho), _ptr(q),
                           _stream_ptr(stream)), "stmg_create")
    return h.value


def stmg_set_field(h: int, field) -> int:
    return _check(lib.stmg_set_field(h, _ptr(field)), "stmg_set_field")


def stmg_set_design(h: int, rho) -> int:
    return _check(lib.stmg_set_design(h, _ptr(rho)), "stmg_set_design")


def stmg_solve_forward(h: int, rhs, u0, u, stats: stmg_stats | None = None) -> int:
    return _check(lib.stmg_solve_forward(h, _ptr(rhs), _ptr(u0), _ptr(u),
                                         C.byref(stats) if stats is not None else None),
                  "stmg_solve_forward")


def stmg_solve_adjoint(h: int, rhs, l0, lam, stats: stmg_stats | None = None) -> int:
    return _check(lib.stmg_solve_adjoint(h, _ptr(rhs), _ptr(l0), _ptr(lam),
                                         C.byref(stats) if stats is not None else None),
                  "stmg_solve_adjoint")


def stmg_objective(h: int, u) -> float:
    out = C.c_double()
    _check(lib.stmg_objective(h, _ptr(u), C.byref(out)), "stmg_objective")
    return out.value


def stmg_gradient(h: int, u, lam, grad) -> int:
    return _check(lib.stmg_gradient(h, _ptr(u), _ptr(lam), _ptr(grad)), "stmg_gradient")


def stmg_gradient_noalloc(problem: stmg_problem, rho, u, lam, grad, stream=None) -> int:
    return _check(lib.stmg_gradient_noalloc(C.byref(problem), _ptr(rho), _ptr(u), _ptr(lam),
                                            _ptr(grad), _stream_ptr(stream)),
                  "stmg_gradient_noalloc")


def stmg_oc_update(h: int, rho, grad, volume: float, move: float, eta: float, rho_min: float,
                   rho_new) -> int:
    return _check(lib.stmg_oc_update(h, _ptr(rho), _ptr(grad), volume, move, eta, rho_min,
                                     _ptr(rho_new)), "stmg_oc_update")


def stmg_get_info(h: int) -> stmg_info:
    info = stmg_info()
    _check(lib.stmg_get_info(h, C.byref(info)), "stmg_get_info")
    return info


def stmg_destroy(h: int) -> int:
    return _check(lib.stmg_destroy(h), "stmg_destroy")


def stmg_level_apply(h, level, transpose, x, y):
    return _check(lib.stmg_level_apply(h, level, int(transpose), _ptr(x), _ptr(y)), "stmg_level_apply")


def stmg_level_smooth(h, level, transpose, nu, b, u):
    return _check(lib.stmg_level_smooth(h, level, int(transpose), nu, _ptr(b), _ptr(u)),
                  "stmg_level_smooth")


def stmg_level_presmooth_restrict(h, level, transpose, nu, b, u, bc):
    return _check(lib.stmg_level_presmooth_restrict(h, level, int(transpose), nu, _ptr(b), _ptr(u),
                                                    _ptr(bc)), "stmg_level_presmooth_restrict")


def stmg_level_prolong_postsmooth(h, level, transpose, nu, b, z, u):
    return _check(lib.stmg_level_prolong_postsmooth(h, level, int(transpose), nu, _ptr(b), _ptr(z),
                                                    _ptr(u)), "stmg_level_prolong_postsmooth")


def stmg_level_coarsest_solve(h, transpose, b, z):
    return _check(lib.stmg_level_coarsest_solve(h, int(transpose), _ptr(b), _ptr(z)),
                  "stmg_level_coarsest_solve")


def stmg_vcycle(h, transpose, b, u) -> float:
    r = C.c_double()
    _check(lib.stmg_vcycle(h, int(transpose), _ptr(b), _ptr(u), C.byref(r)), "stmg_vcycle")
    return r.value


def stmg_pass_geometry(n_el: int, n_t: int, sweeps: int, fp32: bool = False,
                       fine: bool = False) -> dict:
    out = [C.c_int() for _ in range(4)]
    _check(lib.stmg_pass_geometry(n_el, n_t, sweeps, int(fp32), int(fine),
                                  *[C.byref(o) for o in out]), "stmg_pass_geometry")
    return dict(zip(("strip_cols", "strips", "seg_rows", "waves"), (o.value for o in out)))


def stmg_stream_calibrate(a, b, s: float, y, nontemporal: bool = True, stream=None) -> int:
    """Queue y = a (b None) or y = a + s b on `stream` (default: the current stream)."""
    return _check(lib.stmg_stream_calibrate(_ptr(a), _ptr(b), s, _ptr(y), y.numel(),
                                            int(nontemporal), _stream_ptr(stream)),
                  "stmg_stream_calibrate")


# ---- convenience wrapper -------------------------------------------------------------

@dataclass
class Problem:
    """Physical problem; the defaults are the non-dimensional rod x in [0, 1],
    t in [0, 0.1], k = kappa_min + rho^3 (1 - kappa_min), c = 1, q = 1."""
    n_el: int
    n_t: int
    length: float = 1.0
    t_final: float = 0.1
    k_ins: float = 1e-3
    k_con: float = 1.0
    c_ins: float = 1.0
    c_con: float = 1.0
    p_k: float = 3.0
    p_c: float = 2.0
    theta_ref: float = 1.0
    q_uniform: float = 1.0
    field_kind: int = STMG_FIELD_DENSITY

    def c_struct(self) -> stmg_problem:
        return stmg_problem(self.n_el, self.n_t, self.length, self.t_final, self.k_ins,
                            self.k_con, self.c_ins, self.c_con, self.p_k, self.p_c,
                            self.theta_ref, self.q_uniform, self.field_kind)


def make_options(**kw) -> stmg_options:
    o = stmg_default_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class SolveStats:
    status: int
    cycles: int
    n_levels: int
    rel_residual: float
    conv_factor: float
    solve_ms: float
    dof_updates: float
    fine_kernel_ms: float
    fine_kernel_bytes: float
    fine_kernel_launches: int
    fine_passes: int = 0
    setup_ms: float = 0.0
    path: str = ""
    history: list = field(default_factory=list)
    level_cycles: int = 0
    level_ms: list = field(default_factory=list)   # per level, time_levels > 0

    @classmethod
    def from_c(cls, s: stmg_stats) -> "SolveStats":
        n = s.cycles
        return cls(s.status, s.cycles, s.n_levels, s.rel_residual, s.conv_factor, s.solve_ms,
                   s.dof_updates, s.fine_kernel_ms, s.fine_kernel_bytes, s.fine_kernel_launches,
                   s.fine_passes, s.setup_ms, s.path.decode(),
                   [s.history[i] for i in range(n + 1)], s.level_cycles,
                   [s.level_ms[i] for i in range(s.n_levels)] if s.level_cycles else [])


class Solver:
    """Owns one libstmg handle (hierarchy resident on the device).

    Every library call runs on the handle's stream (``stream``, else the stream current
    at construction).  Before each call that stream waits for the work already queued
    on the caller's current stream (which may still be producing an input), and the
    outputs this class allocates are allocated while the handle's stream is current, so
    the caching allocator never hands the library a block that other streams' pending
    work still uses."""

    def __init__(self, problem: Problem, rho, q=None, stream=None, **options):
        import torch
        self._torch = torch
        self.problem = problem
        self.options = make_options(**options)
        self.device = rho.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._event = torch.cuda.Event()      # reused: recorded, then waited on at once
        self._order()
        self.handle = stmg_create(problem.c_struct(), self.options, rho, q, self.stream)

    def _order(self):
        """Make the handle's stream wait for the caller's current stream."""
        cur = self._torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self._event.record(cur)
            self.stream.wait_event(self._event)

    def close(self):
        if getattr(self, "handle", None):
            stmg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.problem.n_t + 1, self.problem.n_el + 1)

    def info(self) -> dict:
        i = stmg_get_info(self.handle)
        n = i.n_levels
        return {"n_levels": n, "n_el": list(i.n_el[:n]), "n_t": list(i.n_t[:n]),
                "h": list(i.h[:n]), "tau": list(i.tau[:n]), "w_diri": list(i.w_diri[:n]),
                "lambda_eff": list(i.lambda_eff[:max(n - 1, 0)]), "path": i.path.decode(),
                "device_bytes": i.device_bytes, "tail_level": i.tail_level}

    def _new(self, shape=None):
        """Output tensor allocated on the handle's stream."""
        with self._torch.cuda.stream(self.stream):
            return self._torch.empty(shape or self.shape, dtype=self._torch.float64,
                                     device=self.device)

    def solve_forward(self, rhs=None, u0=None, out=None):
        u = out if out is not None else self._new()
        st = stmg_stats()
        self._order()
        stmg_solve_forward(self.handle, rhs, u0, u, st)
        return u, SolveStats.from_c(st)

    def solve_adjoint(self, rhs=None, l0=None, out=None):
        lam = out if out is not None else self._new()
        st = stmg_stats()
        self._order()
        stmg_solve_adjoint(self.handle, rhs, l0, lam, st)
        return lam, SolveStats.from_c(st)

    def objective(self, u) -> float:
        self._order()
        return stmg_objective(self.handle, u)

    def gradient(self, u, lam, out=None):
        g = out if out is not None else self._new((self.problem.n_el,))
        self._order()
        stmg_gradient(self.handle, u, lam, g)
        return g

    def set_field(self, field):
        self._order()
        stmg_set_field(self.handle, field)

    def set_design(self, rho):
        self.set_field(rho)

    def oc_update(self, rho, grad, volume: float, move: float = 0.2, eta: float = 0.5,
                  rho_min: float = 1e-3, out=None):
        new = out if out is not None else self._new(tuple(rho.shape))
        self._order()
        stmg_oc_update(self.handle, rho, grad, volume, move, eta, rho_min, new)
        return new


def rel_err(a, b) -> float:
    """max|a - b| / max|b| (norm-wise relative error)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


__all__ = [n for n in dir() if n.startswith("stmg_")] + [
    "Problem", "Solver", "SolveStats", "make_options", "StmgError", "EXPORTED", "lib", "rel_err"]
