"""Continuous-batching request loop for STMG solves on one GPU.

Requests (grid, density field, kappa_min, forward-only or forward + adjoint +
gradient) arrive at any time.  A fixed number of slots, each a host thread with its
own HIP stream, pull requests from the queue as soon as the slot is free and the
request's device footprint (stmg_footprint: the hierarchy and the request's output
vectors) fits the HBM budget; admitted requests run concurrently, so their kernels
overlap on the device.
Hierarchies stay resident after a request: a later request of the same grid and
material re-assembles the idle hierarchy from its density (stmg_set_design, with the
field-independent coarsening path of Section 7.2) instead of allocating a new one.
Idle hierarchies are evicted, least recently used first, when memory is needed.

Recovery: a mixed-precision solve that diverges (FP32 range or rounding can break
the inner cycles where FP64 would not, cf. the divergence bound of Section 3.1) is
solved once more on an FP64 hierarchy built for the request; the extra device memory
is admitted like a request (waiting for releases), and the result records the retry.

All arithmetic runs in libstmg; every kernel is deterministic and independent of
co-running work, so a result does not depend on the mix it was solved in.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class SolveRequest:
    n_el: int
    n_t: int
    rho: np.ndarray
    kappa_min: float = 1e-3
    with_adjoint: bool = False
    rid: int = -1
    length: float = 1.0
    t_final: float = 0.1
    arrival: float = 0.0          # set by Server.submit (perf_counter seconds)

    @property
    def dofs(self) -> int:
        return (self.n_el + 1) * (self.n_t + 1)

    def key(self):
        return (self.n_el, self.n_t, self.kappa_min, self.length, self.t_final)


@dataclass
class SolveResult:
    rid: int
    theta: float
    final_temperature: np.ndarray          # T(x, t_T) on the nodes
    gradient: np.ndarray | None
    forward: B.SolveStats
    adjoint: B.SolveStats | None
    arrival: float
    admitted: float
    completed: float
    slot: int
    reused_hierarchy: bool
    fp64_retry: bool = False            # the mixed solve diverged and FP64 solved it

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class Admission:
    """Admission policy: first come, first served, with backfilling.

    The oldest waiting request is admitted when its footprint fits the free budget;
    otherwise the next waiting requests that fit are admitted ahead of it, unless the
    oldest has been passed over ``max_bypass`` times (then the queue waits for memory,
    so a large request is not starved).  A request larger than the whole budget is
    rejected.
    """

    def __init__(self, budget: int, max_bypass: int = 64):
        self.budget = int(budget)
        self.max_bypass = max_bypass
        self.bypassed = 0

    def pick(self, waiting: list, free: int, footprint) -> int | None:
        """Index into ``waiting`` of the request to admit now, or None."""
        for i, req in enumerate(waiting):
            need = footprint(req)
            if need <= free:
                if i == 0:
                    self.bypassed = 0
                else:
                    if self.bypassed >= self.max_bypass:
                        return None
                    self.bypassed += 1
                return i
        return None


@dataclass
class ServerStats:
    submitted: int = 0
    completed: int = 0
    rejected: int = 0
    reused: int = 0
    created: int = 0
    evicted: int = 0
    retried_fp64: int = 0
    peak_in_flight: int = 0
    peak_bytes: int = 0
    dof_updates: float = 0.0
    latencies: list = field(default_factory=list)


class Server:
    """Continuous batching of STMG solves (see the module docstring)."""

    def __init__(self, device=None, slots: int = 8, hbm_budget: int | None = None,
                 precision: int = B.STMG_MIXED, keep_resident: bool = True,
                 retry_fp64: bool = True, mixed_overrides: dict | None = None, **options):
        """mixed_overrides: options applied to the mixed-precision attempt only (for
        example a tight divergence bound that forces the FP64 retry in a test)."""
        import torch
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda:0")
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.admission = Admission(hbm_budget)
        self.options = dict(options, precision=precision, deff_mode=1)
        self.fp64_options = dict(self.options, precision=B.STMG_FP64)
        if precision == B.STMG_MIXED and mixed_overrides:
            self.options.update(mixed_overrides)
        self.retry_fp64 = retry_fp64 and precision == B.STMG_MIXED
        self._growing = 0                      # in-flight requests waiting for retry memory
        self.keep_resident = keep_resident
        self.stats = ServerStats()
        self._cv = threading.Condition()
        self._waiting: list = []
        self._futures: dict = {}
        self._in_use = 0                       # bytes of admitted requests
        self._in_flight = 0
        self._idle: collections.OrderedDict = collections.OrderedDict()   # id -> (key, solver, bytes)
        self._idle_bytes = 0
        self._closing = False
        self._next_id = 0
        # every slot stream keeps the default priority
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self._threads = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                         for i in range(slots)]
        for t in self._threads:
            t.start()

    # ---- public -------------------------------------------------------------------

    def submit(self, req: SolveRequest) -> Future:
        fut: Future = Future()
        with self._cv:
            if req.rid < 0:
                req.rid = self._next_id
            self._next_id = max(self._next_id, req.rid) + 1
            req.arrival = time.perf_counter()
            self.stats.submitted += 1
            if self._footprint(req) > self.admission.budget:
                self.stats.rejected += 1
                fut.set_exception(MemoryError(
                    f"request {req.rid} needs {self._footprint(req)} bytes, budget "
                    f"{self.admission.budget}"))
                return fut
            self._waiting.append(req)
            self._futures[req.rid] = fut
            self._cv.notify_all()
        return fut

    def close(self):
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        for _, (_, solver, _) in list(self._idle.items()):
            solver.close()
        self._idle.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- internals ----------------------------------------------------------------

    def _problem(self, req: SolveRequest) -> B.Problem:
        return B.Problem(req.n_el, req.n_t, req.length, req.t_final, k_ins=req.kappa_min)

    def _footprint(self, req: SolveRequest, options: dict | None = None) -> int:
        """Device bytes of the request: hierarchy plus outputs (stmg_footprint)."""
        return B.stmg_footprint(self._problem(req).c_struct(),
                                B.make_options(**(options or self.options)), req.with_adjoint)

    @staticmethod
    def _outputs(req: SolveRequest) -> int:
        """The output part of stmg_footprint: u, and with the adjoint Lambda and g."""
        return req.dofs * 8 + ((req.dofs + req.n_el) * 8 if req.with_adjoint else 0)

    def _take_idle(self, key):
        for hid, (k, solver, nbytes) in self._idle.items():
            if k == key:
                del self._idle[hid]
                self._idle_bytes -= nbytes
                return solver, nbytes
        return None, 0

    def _evict_for(self, need: int) -> None:
        while self._idle and self.admission.budget - self._in_use - self._idle_bytes < need:
            _, (_, solver, nbytes) = self._idle.popitem(last=False)
            self._idle_bytes -= nbytes
            solver.close()
            self.stats.evicted += 1

    def _admit(self):
        """Called with the lock held: returns (request, reused solver or None, bytes)."""
        if not self._waiting:
            return None
        # every idle hierarchy, a reusable one included, can be evicted, so a request
        # fits when its whole footprint fits beside the requests in flight
        i = self.admission.pick(self._waiting, self.admission.budget - self._in_use,
                                self._footprint)
        if i is None:
            return None
        req = self._waiting.pop(i)
        solver, _ = self._take_idle(req.key())
        total = self._footprint(req)
        self._evict_for(total)
        self._in_use += total
        self._in_flight += 1
        self.stats.peak_in_flight = max(self.stats.peak_in_flight, self._in_flight)
        self.stats.peak_bytes = max(self.stats.peak_bytes, self._in_use + self._idle_bytes)
        return req, solver, total

    def _worker(self, slot: int):
        torch = self.torch
        stream = self._streams[slot]
        while True:
            with self._cv:
                got = None
                while got is None:
                    if self._closing and not self._waiting:
                        return
                    got = self._admit()
                    if got is None:
                        self._cv.wait(timeout=0.05)
            req, solver, total = got
            admitted = time.perf_counter()
            fut = self._futures.pop(req.rid)
            reused = solver is not None
            try:
                with torch.cuda.stream(stream):
                    rho = torch.from_numpy(np.ascontiguousarray(req.rho, dtype=np.float64)).to(
                        self.device, non_blocking=False)
                    if solver is None:
                        solver = B.Solver(self._problem(req), rho, stream=stream, **self.options)
                        created = True
                    else:
                        solver.set_design(rho)
                        created = False
                    u, fst = solver.solve_forward()
                    retried = False
                    if fst.status == B.STMG_DIVERGED and self.retry_fp64:
                        solver, total, u, fst = self._fp64_retry(req, solver, total, rho)
                        retried = True
                    theta = solver.objective(u)
                    grad, ast = None, None
                    if req.with_adjoint:
                        lam, ast = solver.solve_adjoint()
                        grad = solver.gradient(u, lam).cpu().numpy()
                        del lam
                    final = u[-1].cpu().numpy()
                    del u, rho
                    stream.synchronize()
                done = time.perf_counter()
                res = SolveResult(req.rid, theta, final, grad, fst, ast, req.arrival, admitted,
                                  done, slot, reused, retried)
                with self._cv:
                    self.stats.completed += 1
                    self.stats.reused += int(reused)
                    self.stats.retried_fp64 += int(retried)
                    self.stats.created += int(created)
                    self.stats.dof_updates += fst.dof_updates + (ast.dof_updates if ast else 0.0)
                    self.stats.latencies.append(res.latency)
                    self._release(req, solver, total)
                fut.set_result(res)
            except Exception as exc:  # the request fails, the server keeps going
                with self._cv:
                    self._release(req, solver, total, keep=False)
                fut.set_exception(exc)

    def _fp64_retry(self, req, solver, total, rho):
        """The mixed solve diverged: drop its hierarchy and solve once in FP64 on a new
        one, admitted for the difference in footprint.  Returns the FP64 solver, the
        request's new byte total, u and the stats."""
        solver.close()
        need = self._footprint(req, self.fp64_options)
        if not self._grow(need - total):
            raise MemoryError(f"request {req.rid}: no memory for the FP64 retry ({need} bytes)")
        try:
            fp64 = B.Solver(self._problem(req), rho, stream=solver.stream, **self.fp64_options)
        except Exception:
            self._grow(total - need)           # hand the extra bytes back
            raise
        fp64.fp64_retry = True
        u, fst = fp64.solve_forward()
        return fp64, need, u, fst

    def _grow(self, extra: int) -> bool:
        """Admit `extra` more bytes for a request in flight, waiting for releases and
        evicting idle hierarchies; gives up when every request in flight is waiting too."""
        if extra <= 0:
            with self._cv:
                self._in_use += extra
            return True
        with self._cv:
            self._growing += 1
            try:
                while True:
                    self._evict_for(extra)
                    if self.admission.budget - self._in_use - self._idle_bytes >= extra:
                        self._in_use += extra
                        self.stats.peak_bytes = max(self.stats.peak_bytes,
                                                    self._in_use + self._idle_bytes)
                        return True
                    if self._in_flight - self._growing <= 0:
                        return False
                    self._cv.wait(timeout=0.05)
            finally:
                self._growing -= 1

    def _release(self, req, solver, total, keep=True):
        """Lock held: return the request's memory; keep its hierarchy resident."""
        self._in_use -= total
        self._in_flight -= 1
        if getattr(solver, "fp64_retry", False):
            keep = False                       # FP64 hierarchies do not serve later requests
        if solver is not None and keep and self.keep_resident:
            hb = total - self._outputs(req)
            self._idle[id(solver)] = (req.key(), solver, hb)
            self._idle_bytes += hb
        elif solver is not None:
            solver.close()
        self._cv.notify_all()


def percentiles(xs, qs=(50, 99)):
    a = np.asarray(xs, dtype=np.float64)
    return {f"p{q}": float(np.percentile(a, q)) for q in qs} if a.size else {}
