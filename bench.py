"""Benchmark of the STMG hot path on one MI355X.

Default workload: boxfilt_8192x65536 (8192 elements x 65536 steps, 5.4e8 space-time
DOFs, box-filtered uniform densities, kappa_min = 1e-4), FP64, V(2,2) cycles to the
1e-10 relative residual: the largest configuration, the one that is bound by HBM.

One step = one pass of the whole path on a device-resident design field:
re-assemble every level from rho (SIMP, Algorithm 3 decision, R-averaged coarse
operators), forward STMG solve to the relative-residual tolerance, adjoint STMG solve,
objective and gradient.  Reported value: DOF-updates/s = (sum over both solves of
cycles * sum_{l < N_l} 2 nu n_l) / wall time of the K timed steps.  Beside it: the
mixed-precision forward solve of the same input (time to the same FP64 residual),
the fine-level kernel's achieved bandwidth against the HBM peak, the device's streaming
rates from plain HIP copy and triad kernels, and the CPU oracle on a bounded sample.

Prints ONE JSON line (rank 0).  --gpus above 1 is rejected: the path runs on one GPU (the
library has no multi-GPU form).
"""
from __future__ import annotations

import argparse
from concurrent.futures import ThreadPoolExecutor
import json
import os
import subprocess
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

METRIC = "STMG DOF-updates/s + % HBM roofline; p50/p99 solve latency at 1e-10 resid"
HBM_PEAK_GBS = 8000.0

# Workloads: name -> (nu, concurrent solves by default).  nu = 2 unless V(2,2) fails
# to converge within the cycle cap, then the paper's default nu = 5.  The forward and
# adjoint solves of a step run concurrently where the levels are small enough for one
# solve's latency-bound launches to leave the device idle; on the HBM-bound
# configuration they run one after the other (each saturates HBM alone).
WORKLOADS = {
    "uniform_64x64": (2, True),
    "block_1024x4096": (5, True),
    "block_2048x8192": (5, True),
    "boxfilt_8192x65536": (2, False),
}
DEFAULT_WORKLOAD = "boxfilt_8192x65536"
# the oracle samples at most this many DOFs (the leading time steps of the workload)
CPU_SAMPLE_DOFS = 4_300_000


# The fine passes of every TIMED_EVERY-th V-cycle are bracketed by HIP events: enough
# launches for the average, without an event marker between every pair of kernels.
TIMED_EVERY = 8


def measured_traffic(workload: str):
    """Per-launch HBM bytes of the fine-level passes from the committed counter runs,
    or None when the kernel sources changed since they were taken."""
    import hashlib
    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    data = json.loads(path.read_text())
    csrc = ROOT / "paper_2505_10168_amd" / "csrc"
    digest = hashlib.sha256((csrc / "kernels_fused.hip").read_bytes() +
                            (csrc / "stmg_device.hpp").read_bytes()).hexdigest()
    if digest != data.get("src_sha256"):
        return None
    entry = data.get("workloads", {}).get(workload)
    return entry["bytes_per_launch"] if entry else None


def stream_rates(dev, nbytes: int = 2 << 30, reps: int = 10) -> dict:
    """Streaming rates of this device from the library's plain HIP kernels on 2 GiB FP64
    vectors, (bytes read + written) / time: a copy (1 read, 1 write stream) and a triad
    (2 reads, 1 write), with non-temporal stores as the fused passes use and without;
    torch's copy_ beside them.  The practical ceiling the fine pass is compared with."""
    import torch

    from paper_2505_10168_amd import binding as B
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.full_like(a, 2.0)
    y = torch.empty_like(a)
    st = torch.cuda.current_stream(dev)
    out = {}

    def timed(fn, moved):
        for _ in range(2):
            fn()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(st)
        for _ in range(reps):
            fn()
        t1.record(st)
        torch.cuda.synchronize()
        return moved / (t0.elapsed_time(t1) / reps * 1e-3) / 1e9

    for nt in (True, False):
        tag = "_nt" if nt else ""
        out["copy" + tag] = timed(lambda: B.stmg_stream_calibrate(a, None, 0.0, y, nt, st),
                                  2 * nbytes)
        out["triad" + tag] = timed(lambda: B.stmg_stream_calibrate(a, b, 0.5, y, nt, st),
                                   3 * nbytes)
    out["torch_copy"] = timed(lambda: y.copy_(a), 2 * nbytes)
    del a, b, y
    torch.cuda.empty_cache()
    return {k: round(v, 1) for k, v in out.items()}


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else float("nan")


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload: str, nu: int, budget_s: float) -> dict:
    """Time the oracle's forward V-cycles on the workload's input in child processes,
    for about budget_s seconds each: once with every BLAS/OpenMP pool pinned to one
    thread and once allowed all of the host's threads.  Workloads above CPU_SAMPLE_DOFS
    are sampled: the same field, h and tau over the leading time steps only."""
    w_dofs = None
    try:
        from paper_2505_10168_amd import inputs as I
        w = I.workload(workload)
        w_dofs = w.dofs
        # a power of two of leading steps keeps the sample's time axis halvable
        n_t = w.n_t if w.dofs <= CPU_SAMPLE_DOFS else \
            1 << max(1, int(np.log2(CPU_SAMPLE_DOFS / (w.n_el + 1))))
    except Exception:
        n_t = None
    runs = {}
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    for threads in (1, nproc):
        runs[threads] = _cpu_run(workload, nu, budget_s, n_t, threads)
    one = runs[1]
    if one.get("error"):
        return {"value": None, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
                "sample": f"failed: {one['error']}"}
    many = runs[nproc]
    sampled = n_t is not None and w_dofs is not None and n_t != w.n_t
    what = (f"the first {n_t} of {w.n_t} time steps of {workload} (same field, h and tau; "
            f"{(w.n_el + 1) * (n_t + 1):.3g} of {w_dofs:.3g} DOFs)" if sampled else workload)
    return {
        "value": one["dof_updates"] / one["seconds"], "unit": "DOF-updates/s", "cores": 1,
        "kind": "oracle",
        "sample": f"{one['cycles']} forward V-cycles (nu={nu}) of the NumPy FP64 oracle on "
                  f"{what}, {one['seconds']:.1f} s; hierarchy setup {one['setup_s']:.1f} s "
                  f"excluded",
        "all_threads": {"threads_allowed": nproc,
                        "value": (many["dof_updates"] / many["seconds"]) if not many.get("error")
                        else None,
                        "cycles": many.get("cycles")},
        "nproc": nproc, "cpu_model": cpu_model(),
        "note": "the oracle's NumPy/SciPy kernels run on one thread whatever the pool size",
    }


def _cpu_run(workload: str, nu: int, budget_s: float, n_t, threads: int) -> dict:
    code = f"""
import os, sys, time, json
sys.path.insert(0, {str(ROOT)!r})
import numpy as np
import oracle as O
from paper_2505_10168_amd import inputs as I
w = I.workload({workload!r})
n_t = {n_t!r} or w.n_t
mat = O.Material(w.kappa_min, 1.0, 1.0, 1.0)
lv = O.make_fine_level(w.rho, mat, n_t, w.length, w.t_final * n_t / w.n_t)
t0 = time.perf_counter()
h = O.build_hierarchy(lv, O.Options(nu={nu}))
b = O.load_vector(lv, 1.0)
setup = time.perf_counter() - t0
u = np.zeros(lv.shape)
per_cycle = sum(2 * {nu} * O.dofs(l) for l in h.levels[:-1])
t0 = time.perf_counter(); n = 0
while True:
    u = O.vcycle(h, 0, u, b)
    n += 1
    el = time.perf_counter() - t0
    if el > {budget_s} or n >= 200:
        break
print(json.dumps({{"cycles": n, "seconds": el, "dof_updates": n * per_cycle, "setup_s": setup}}))
"""
    t = str(threads)
    env = dict(os.environ, OMP_NUM_THREADS=t, OPENBLAS_NUM_THREADS=t, MKL_NUM_THREADS=t)
    try:
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             env=env, timeout=max(600, 20 * budget_s))
    except subprocess.TimeoutExpired:
        return {"error": "timed out"}
    if out.returncode != 0:
        return {"error": out.stderr[-300:]}
    return json.loads(out.stdout.strip().splitlines()[-1])


def serving_bench(args):
    """Configuration 5: a Poisson stream of solve requests at 0.7 x the closed-loop
    rate of a warm-up burst; mixed precision to 1e-10; half forward-only, half forward
    + adjoint + gradient.  Latency = completion - arrival."""
    import threading

    import torch

    from paper_2505_10168_amd import inputs as I
    from paper_2505_10168_amd.serving import Server, SolveRequest, percentiles

    dev = torch.device("cuda:0")
    n = args.serving

    def reqs(rate):
        return [SolveRequest(r.n_el, r.n_t, r.rho, r.kappa_min, r.with_adjoint, rid=r.rid)
                for r in I.request_stream(n, rate, seed=5)]

    # nu = 20: at kappa_min = 1e-4 the block fields stall at nu = 5 (factors 0.93-1.0)
    opts = dict(nu=args.nu if args.nu is not None else 20, max_cycles=300)
    with Server(dev, slots=args.slots, **opts) as srv:
        warm = reqs(1.0)[: args.serving_warmup]
        t0 = time.perf_counter()
        for f in [srv.submit(r) for r in warm]:
            f.result()
        closed = len(warm) / (time.perf_counter() - t0)
        rate = 0.7 * closed
        stream = I.request_stream(n, rate, seed=5)
        todo = reqs(rate)
        base = srv.stats.dof_updates
        futs = []
        start = time.perf_counter()

        def feeder():
            for r, meta in zip(todo, stream):
                delay = start + meta.arrival_s - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                futs.append(srv.submit(r))

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        results = [f.result() for f in futs]
        end = max(r.completed for r in results)
        lat = [1e3 * r.latency for r in results]
        p = percentiles(lat)
        out = {
            "metric": METRIC,
            "value": p["p50"],
            "unit": "ms (p50 latency)",
            "n_gpus": 1,
            "steps": n,
            "warmup": len(warm),
            "ms_per_step": 1e3 * (end - start) / n,
            "higher_is_better": False,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64+f32",
            "data": "synthetic",
            "config": {"workload": f"poisson_{n}_requests", "arrival_rate_per_s": rate,
                       "closed_loop_solves_per_s": closed, "slots": args.slots,
                       "precision": "mixed", "tol": 1e-10, **opts},
            "latency_ms": {**p, "max": max(lat)},
            "solves_per_s": n / (end - start),
            "dof_updates_per_s": (srv.stats.dof_updates - base) / (end - start),
            "non_converged": sum(1 for r in results if r.forward.status != 0 or
                                 (r.adjoint is not None and r.adjoint.status != 0)),
            "peak_in_flight": srv.stats.peak_in_flight,
            "hierarchies_created": srv.stats.created,
            "hierarchies_reused": srv.stats.reused,
        }
    print(json.dumps(out), flush=True)


def design_bench(args):
    """The optimisation problem of Section 7 (problem 7's rod and materials, the
    many-frequency load, volume <= 1/2, chi = 1/2 at the start; nu = 20, six levels)
    run on one resident hierarchy until Theta changes by less than 0.1 % for five
    consecutive cycles: forward and adjoint solves concurrently, the gradient, the
    optimality-criteria update and the re-assembly per cycle."""
    import torch

    from paper_2505_10168_amd.design import SECTION7_OPTIONS, DesignLoop, section7_problem

    dev = torch.device("cuda:0")
    n = args.design
    prob, q = section7_problem(n, n)
    q = torch.as_tensor(q, dtype=torch.float64, device=dev)
    rho0 = torch.full((n,), 0.5, dtype=torch.float64, device=dev)
    # one untimed loop of a few cycles loads the code objects and pinned buffers
    warm = DesignLoop(prob, rho0, 0.5, q=q, warm_start=not args.cold, **SECTION7_OPTIONS)
    warm.run(min(3, args.design_cycles))
    warm.close()
    loop = DesignLoop(prob, rho0, 0.5, q=q, warm_start=not args.cold, **SECTION7_OPTIONS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = loop.run(args.design_cycles)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k = len(h.theta)
    out = {
        "metric": "optimisation cycles/s (Section 7 design loop)",
        "value": k / dt,
        "unit": "cycles/s",
        "n_gpus": 1,
        "steps": k,
        "warmup": min(3, args.design_cycles),
        "ms_per_step": 1e3 * dt / k,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"section7_{n}x{n}", "volume": 0.5,
                   "restarts": "cold" if args.cold else "warm", **SECTION7_OPTIONS},
        "converged": h.converged,
        "theta_first": h.theta[0],
        "theta_final": h.theta[-1],
        "stmg_cycles": {"forward_mean": sum(h.forward_cycles) / k,
                        "forward_max": max(h.forward_cycles),
                        "adjoint_mean": sum(h.adjoint_cycles) / k,
                        "adjoint_max": max(h.adjoint_cycles)},
        "dof_updates_per_s": h.dof_updates / dt,
    }
    loop.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--nu", type=int, default=None)
    ap.add_argument("--fused", type=int, default=1)
    ap.add_argument("--interp", default="C", choices=["C", "B"],
                    help="interpolation in time: causal (C, the paper's default) or bilinear (B)")
    ap.add_argument("--reassembly", default="R", choices=["R", "K", "D", "P"],
                    help="coarse operators: resistivity (R, default), conductivity (K) or "
                         "design-field (D) averaging, or Galerkin products (P)")
    ap.add_argument("--no-adjoint", action="store_true")
    conc = ap.add_mutually_exclusive_group()
    conc.add_argument("--sequential", action="store_true",
                      help="run the forward and adjoint solves of a step one after the other "
                           "on one handle")
    conc.add_argument("--concurrent", action="store_true",
                      help="run them concurrently, one handle, stream and host thread each")
    ap.add_argument("--mixed-solves", type=int, default=3,
                    help="timed mixed-precision forward solves of the same input (0: none)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving", type=int, default=0,
                    help="run the serving workload with this many requests instead")
    ap.add_argument("--serving-warmup", type=int, default=32)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--design", type=int, default=0,
                    help="run the Section 7 design loop on an N x N grid instead")
    ap.add_argument("--design-cycles", type=int, default=200)
    ap.add_argument("--cold", action="store_true", help="design loop with cold restarts")
    ap.add_argument("--timed-every", type=int, default=TIMED_EVERY,
                    help="time the fine passes of every k-th V-cycle with HIP events")
    ap.add_argument("--no-levels", action="store_true",
                    help="skip the level-by-level timing of one forward solve")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the STMG path runs on one GPU only (the library has no multi-GPU "
              "form); --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    if args.serving:
        serving_bench(args)
        return
    if args.design:
        design_bench(args)
        return

    import torch

    from paper_2505_10168_amd import binding as B
    from paper_2505_10168_amd import inputs as I

    dev = torch.device("cuda:0")
    w = I.workload(args.workload)
    nu_default, conc_default = WORKLOADS[args.workload]
    nu = args.nu if args.nu is not None else nu_default
    precision = B.STMG_MIXED if args.precision == "mixed" else B.STMG_FP64
    prob = B.Problem(w.n_el, w.n_t, w.length, w.t_final, k_ins=w.kappa_min)
    rho = torch.from_numpy(w.rho).to(dev)
    # The adjoint right-hand side does not depend on u, so a step's two solves are
    # independent and may run concurrently, each on its own handle, stream and thread.
    concurrent = (args.concurrent or (conc_default and not args.sequential)) and not args.no_adjoint
    s_fwd = torch.cuda.Stream(device=dev) if concurrent else None
    s_adj = torch.cuda.Stream(device=dev) if concurrent else None
    opts = dict(nu=nu, precision=precision, fused=args.fused, time_kernels=args.timed_every,
                interp=B.STMG_INTERP_B if args.interp == "B" else B.STMG_INTERP_C,
                reassembly="RKDP".index(args.reassembly))
    solver = B.Solver(prob, rho, stream=s_fwd, **opts)
    adj_solver = B.Solver(prob, rho, stream=s_adj, **opts) if concurrent else solver
    pool = ThreadPoolExecutor(max_workers=2) if concurrent else None
    info = solver.info()
    u = solver._new()
    lam = adj_solver._new()
    grad = solver._new((w.n_el,))

    def forward():
        solver.set_design(rho)
        return solver.solve_forward(out=u)[1]

    def adjoint():
        if adj_solver is not solver:
            adj_solver.set_design(rho)
        return adj_solver.solve_adjoint(out=lam)[1]

    def step(record):
        if concurrent:
            fa, fb = pool.submit(forward), pool.submit(adjoint)
            rec = {"fwd": fa.result(), "adj": fb.result()}
        else:
            rec = {"fwd": forward()}
            if not args.no_adjoint:
                rec["adj"] = adjoint()
        if not args.no_adjoint:
            solver.gradient(u, lam, out=grad)
        rec["theta"] = solver.objective(u)
        record.append(rec)

    warm = []
    for _ in range(args.warmup):
        step(warm)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    solves = [r[k] for r in recs for k in ("fwd", "adj") if k in r]
    dof_updates = sum(s.dof_updates for s in solves)
    lat = [s.solve_ms for s in solves]
    kern_ms = sum(s.fine_kernel_ms for s in solves)
    kern_bytes = sum(s.fine_kernel_bytes for s in solves)
    launches = sum(s.fine_kernel_launches for s in solves)
    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    # share of the solves' wall time spent in fine-level passes (all of them, from the
    # average of the timed ones)
    avg_us = 1e3 * kern_ms / launches if launches else None
    fine_share = (sum(s.fine_passes for s in solves) * avg_us * 1e-3 / sum(lat)
                  if avg_us and precision == B.STMG_FP64 else None)
    bad = [s.status for s in solves if s.status != 0]

    fwd_ms = [r["fwd"].solve_ms for r in recs]
    mixed = None
    if args.mixed_solves and precision == B.STMG_FP64:
        # the same forward solve in mixed precision on the same input
        msolver = B.Solver(prob, rho, **dict(opts, precision=B.STMG_MIXED, time_kernels=0))
        mu = msolver._new()
        msolver.solve_forward(out=mu)
        mst = [msolver.solve_forward(out=mu)[1] for _ in range(args.mixed_solves)]
        mms = [m.solve_ms for m in mst]
        mixed = {"form": "FP32 smoothing and transfers inside FP64 defect correction, "
                         "same input and tolerance",
                 "solve_ms_p50": percentile(mms, 50), "solves": len(mms),
                 "cycles": mst[-1].cycles, "rel_residual": mst[-1].rel_residual,
                 "status": mst[-1].status,
                 "fp64_forward_solve_ms_p50": percentile(fwd_ms, 50),
                 "speedup_vs_fp64": percentile(fwd_ms, 50) / percentile(mms, 50),
                 "dof_updates_per_s": mst[-1].dof_updates / (percentile(mms, 50) * 1e-3)}
        del mu
        msolver.close()
    levels = None
    if not args.no_levels:
        # one more forward solve (outside the timed steps) with events at every level
        # boundary of every cycle: where a cycle's device time goes
        lsolver = B.Solver(prob, rho, **dict(opts, time_kernels=0, time_levels=1))
        _, lst = lsolver.solve_forward(out=u)
        li = lsolver.info()
        levels = {"ms_per_cycle": [round(x, 5) for x in lst.level_ms],
                  "n_el": li["n_el"], "n_t": li["n_t"], "tail_level": li["tail_level"],
                  "cycles_timed": lst.level_cycles,
                  "sum_ms_per_cycle": sum(lst.level_ms),
                  "solve_ms_per_cycle": lst.solve_ms / max(lst.cycles, 1)}
        lsolver.close()
    solver.close()
    if concurrent:
        adj_solver.close()
        pool.shutdown()
    del u, lam, grad
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rates = stream_rates(dev)
    copy_gbs = rates["copy_nt"]

    out = {
        "metric": METRIC,
        "value": dof_updates / elapsed,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == B.STMG_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "n_el": w.n_el, "n_t": w.n_t, "dofs": w.dofs,
            "kappa_min": w.kappa_min, "nu": nu, "tol": 1e-10, "precision": args.precision,
            "interp": args.interp, "reassembly": args.reassembly,
            "path": info["path"], "levels": info["n_levels"],
            "step": "reassemble + forward solve" + ("" if args.no_adjoint else
                                                  " + adjoint solve + gradient") + " + objective",
            "solves": ("forward and adjoint concurrently, one handle and stream each"
                       if concurrent else "one after the other"),
        },
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "solves": len(lat)},
        "solve": {
            "fwd_cycles": recs[-1]["fwd"].cycles,
            "adj_cycles": recs[-1]["adj"].cycles if "adj" in recs[-1] else None,
            "fwd_rel_residual": recs[-1]["fwd"].rel_residual,
            "adj_rel_residual": recs[-1]["adj"].rel_residual if "adj" in recs[-1] else None,
            "theta": recs[-1]["theta"], "non_converged": len(bad),
            "setup_ms": recs[-1]["fwd"].setup_ms,
        },
        "mixed_precision": mixed,
        "level_breakdown": levels,
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_fused_fine<double, TR, 0, 1, 2, 1, 2, 1> (the finest level's "
                       "cross-cycle pass)" if args.workload == "boxfilt_8192x65536" and nu == 2
                       else "k_fused_fine (the finest level's fused passes)"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(args.workload) if args.precision == "fp64" else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "launches": launches,
            "avg_launch_us": avg_us,
            "bytes_per_launch": kern_bytes / launches if launches else None,
            "share_of_solve_time": fine_share,
            "timed_every_nth_cycle": args.timed_every,
            "stream_GBs": rates,
            "copy_GBs": copy_gbs,
            "copy_frac": (achieved / copy_gbs) if achieved else None,
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, nu, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
