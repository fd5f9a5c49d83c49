"""Times the parallel CPU executor (executor.c) on the benchmark's workloads:
the second CPU baseline of the benchmark, run by it as a child process so
that the OpenMP thread placement (OMP_PROC_BIND=close, OMP_PLACES=cores, set
here before the runtime starts) applies.  BASELINE INFRASTRUCTURE ONLY.

The schedule is GrowLocal (Algorithm 3.1) with one core per host thread and
the paper's parameters (L = 500, alpha0 = 20, growth 1.5, acceptance 0.97),
as the paper schedules for its CPU executor; it is built by the library's
host scheduler, whose schedules equal the oracle's bit for bit (tested).
Every timed solve's x is compared with the serial oracle's.

Usage: python -m oracle.executor_bench --workload er1e7 [--seconds 10]
Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

os.environ.setdefault("OMP_PROC_BIND", "close")
os.environ.setdefault("OMP_PLACES", "cores")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="er1e7", choices=["er1e7"])
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--threads", type=int, default=0, help="0: OMP_NUM_THREADS, else the host's cores")
    args = ap.parse_args()
    import oracle
    from paper_2503_05408_amd import binding as B
    from paper_2503_05408_amd import gen
    threads = args.threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or (os.cpu_count() or 1)
    t = time.perf_counter()
    m = gen.er_n1e7()
    t_gen = time.perf_counter() - t
    t = time.perf_counter()
    core, sup, S = B.schedule(m, B.default_opts(k=threads))
    t_sched = time.perf_counter() - t
    ex = oracle.Executor(m, core, sup)
    b = np.ones(m.n)
    want = oracle.solve(m, b)
    x, used = ex.solve(b, threads)
    exact = oracle.same_bits(x, want)
    reps, t0 = 0, time.perf_counter()
    while True:
        x, used = ex.solve(b, threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= args.seconds or reps >= 200:
            break
    exact = exact and oracle.same_bits(x, want)
    print(json.dumps({
        "value": reps * m.n / el if exact else 0.0, "unit": "rows/s", "cores": used,
        "kind": "bsp_executor_openmp",
        "sample": f"{reps} solves of the full matrix ({el:.1f} s) on {used} threads "
                  f"(OMP_PROC_BIND={os.environ['OMP_PROC_BIND']}, OMP_PLACES={os.environ['OMP_PLACES']})",
        "schedule": f"GrowLocal k={threads} L=500 alpha0=20 (the paper's parameters), S={S}",
        "ms_per_solve": el / reps * 1e3, "exact": bool(exact), "generate_s": t_gen, "schedule_s": t_sched,
    }), flush=True)


if __name__ == "__main__":
    main()
