#!/usr/bin/env python3
"""Benchmark of the GrowLocal-scheduled sparse triangular solve on one MI355X.

One step = one full solve of A x = b (b = all ones, as in the paper's timing
runs) through the persistent kernel: b is read and x written in the original
numbering, every superstep of the schedule runs inside one launch.  The
schedule and the packed device layout are built once before timing (the
paper amortises scheduling over repeated solves with one pattern, Sec. 7.6).

Prints one JSON line.  Rows count only if the GPU result is bitwise equal to
the CPU oracle's (checked before timing).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_2503_05408_amd import gen
    if name == "er1e7":
        n = 10_000_000
        m = gen.erdos_renyi(n, 20.0 / (n - 1), gen.SEED_BASE + 200, name="ER_n1e7_d10")
        desc = ("Erdos-Renyi lower-triangular, n=1e7, 10 off-diagonals/row on average, "
                "values as Sec. 6.2.4 (single system)")
    elif name == "st7":
        m = gen.stencil_3d7(216)
        desc = "3-D 7-point Laplacian lower triangle 216^3 (n=10,077,696)"
    elif name == "st27":
        m = gen.stencil_3d27(216)
        desc = "3-D 27-point Laplacian lower triangle 216^3 (n=10,077,696)"
    elif name == "er1e5":
        m = gen.erdos_renyi_paper(100_000, 1e-4, gen.SEED_BASE)
        desc = "Erdos-Renyi n=1e5 p=1e-4 (q=2p), Table A.4 family"
    else:
        raise SystemExit(f"unknown workload {name}")
    return m, desc


def algorithmic_bytes(n: int, nnz: int) -> int:
    # 12 B per stored entry (8 B value + 4 B index), b read 8 B and x write 8 B per row
    return 12 * nnz + 16 * n


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2503_05408_amd/csrc/gltrsv.hip", "paper_2503_05408_amd/csrc/analysis.cpp",
              "paper_2503_05408_amd/csrc/analysis.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name: str, kernel: str):
    """HBM-side bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated with the copy kernel), or None when no
    summary exists for this workload or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"trsv_{workload_name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources_hash") != kernel_sources_hash() or kernel not in t.get("per_launch", {}):
        return None
    k = t["per_launch"][kernel]
    return k["fetch_bytes"] + k["write_bytes"]


def cpu_baseline(m, budget_s: float = 15.0):
    import oracle
    b = np.ones(m.n)
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.solve(m, b)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    return {"value": reps * m.n / el, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} serial solves of the full matrix ({el:.1f} s), single host thread, "
                      f"{platform.processor() or platform.machine()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="er1e7")
    ap.add_argument("--schedule", default="growlocal", choices=["growlocal", "wavefront"])
    ap.add_argument("--L", type=float, default=50.0)
    ap.add_argument("--alpha0", type=float, default=1.0)
    ap.add_argument("--k", type=int, default=1 << 16)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solve has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_2503_05408_amd import binding as B

    t = time.time()
    m, desc = workload(args.workload)
    log(f"workload {m.name}: n={m.n} nnz={m.nnz} generated in {time.time() - t:.1f} s")
    kind = B.SCHED_WAVEFRONT if args.schedule == "wavefront" else B.SCHED_GROWLOCAL
    opts = B.default_opts(k=args.k, L=args.L, alpha0=args.alpha0, schedule_kind=kind)
    t = time.time()
    plan = B.Plan(m, opts)
    info = plan.info()
    log(f"plan: S={info['supersteps']} wavefronts={info['wavefronts']} chunks={info['chunks']} "
        f"grid={info['grid_blocks']} analysis {info['analysis_ns'] / 1e9:.1f} s (wall {time.time() - t:.1f} s)")

    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()

    # exactness gate
    want = oracle.solve(m, np.ones(m.n))
    plan.solve(b, x)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise SystemExit("device reported an error")
    exact = oracle.same_bits(x.cpu().numpy(), want)
    x.fill_(float("nan"))
    plan.solve_plain(b, x)
    torch.cuda.synchronize()
    exact_plain = oracle.same_bits(x.cpu().numpy(), want)
    log(f"parity: persistent {exact}, plain {exact_plain}")

    for _ in range(args.warmup):
        plan.solve(b, x)
    torch.cuda.synchronize()

    # timed region: K persistent solves, one event pair per solve
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for e0, e1 in evs:
        e0.record(stream)
        plan.solve(b, x)
        e1.record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    per = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    if plan.device_status() != 0:
        raise SystemExit("device reported an error during timing")
    ms = total_ms / args.steps

    # plain: one launch per superstep
    for _ in range(2):
        plan.solve_plain(b, x)
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for _ in range(args.plain_steps):
        plan.solve_plain(b, x)
    p1.record(stream)
    torch.cuda.synchronize()
    ms_plain = p0.elapsed_time(p1) / args.plain_steps

    # achievable copy bandwidth (read + write of 1 GiB) with the library's copy kernel
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    B.copy_probe(src, dst)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        B.copy_probe(src, dst)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    rows_s = m.n / (ms * 1e-3) if exact else 0.0
    rows_s_plain = m.n / (ms_plain * 1e-3) if exact_plain else 0.0
    alg = algorithmic_bytes(m.n, m.nnz)
    kern_ms = float(np.mean(per))
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, "trsv_persistent") if args.schedule == "growlocal" else None
    out = {
        "metric": "reduced elements/sec (exact) at 1 MI355X vs plain launch; p50/p99 latency",
        "value": rows_s,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "n": m.n, "nnz": m.nnz,
            "schedule": f"{args.schedule} k={args.k} L={args.L:g} alpha0={args.alpha0:g}",
            "supersteps": info["supersteps"], "wavefronts": info["wavefronts"],
            "chunks": info["chunks"], "grid_blocks": info["grid_blocks"],
            "analysis_s": info["analysis_ns"] / 1e9,
        },
        "exact": bool(exact and exact_plain),
        "plain": {"value": rows_s_plain, "ms_per_step": ms_plain, "launches_per_step": info["supersteps"]},
        "speedup_vs_plain": (ms_plain / ms) if ms > 0 else None,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "trsv_persistent", "alg_bytes_per_launch": alg, "kernel_ms": kern_ms,
            "copy_probe_GBs": copy_gbs,
            "traffic_GBs": (traffic / (kern_ms * 1e-3) / 1e9) if traffic else None,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(m)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
