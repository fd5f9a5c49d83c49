#!/usr/bin/env python3
"""Benchmark of the GrowLocal-scheduled sparse triangular solve on one MI355X.

One step = one full solve of A x = b (b = all ones, as in the paper's timing
runs) through the persistent kernel: b is read and x written in the original
numbering, every superstep of the schedule runs inside one launch.  The
schedule and the packed device layout are built once before timing (the
paper amortises scheduling over repeated solves with one pattern, Sec. 7.6).

Prints one JSON line.  Rows count only if the GPU result is bitwise equal to
the CPU oracle's (checked before timing).  Besides the headline (the n = 1e7
Erdos-Renyi system) the default line carries:
  c2_st27     the 3-D 27-point 216^3 grid in every single-system form;
  c3_batch    64 systems in one hipGraph launch against 64 plain solves;
  c5_serve    a 10 s Poisson serving run, every result compared bit for bit
              (c5_serve_other_form: the same stream with the server's other
              execution form, BSP or semi-asynchronous);
  third_bound the bound t >= t0 + S t_sync + sum_s max_p w(task) t_entry of
              Sec. 2.3 / Eq. (3.1) with measured constants (and, for the
              semi-asynchronous forms, t0 + levels t_hop), also per key;
  schedule_vs_oracle  the schedule's (pi, sigma, perm) key against the
              oracle's, stored by tests/golden/make_schedule_keys.py;
  cpu_baseline the serial oracle and, as parallel_executor, the schedule run
              on all host threads (oracle/executor.c, the paper's kind of
              CPU executor, Sec. 6.1).
Each roofline object names its kernel and carries, besides the algorithmic
bytes against HBM, the measured traffic and VALU issue of that kernel from
the committed rocprofv3 counters (profiles/*_traffic.json), over this run's
time; both are null once the kernel sources differ from the profiled ones.
"""
from __future__ import annotations

import argparse
import ctypes
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
        m = gen.er_n1e7()
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
    elif name == "nb1e5":
        m = gen.narrow_band(100_000, 0.03, 42.0, gen.SEED_BASE + 10)
        desc = "narrow band n=1e5 p=0.03 B=42, Table A.5 family"
    else:
        raise SystemExit(f"unknown workload {name}")
    return m, desc


def algorithmic_bytes(n: int, nnz: int) -> int:
    # 12 B per stored entry (8 B value + 4 B index), b read 8 B and x write 8 B per row
    return 12 * nnz + 16 * n


def kernel_sources_hash() -> str:
    """Hash of what the measured kernels are built from: the kernels, the
    constants they share with the host, and the analysis that lays out the
    stream they read."""
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2503_05408_amd/csrc/kernels.hip", "paper_2503_05408_amd/csrc/internal.h",
              "paper_2503_05408_amd/csrc/analysis.cpp", "paper_2503_05408_amd/csrc/analysis.h",
              "paper_2503_05408_amd/csrc/wave.cpp", "paper_2503_05408_amd/csrc/wave.h"):
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


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per 4 cycles per SIMD
VALU_PEAK_INSTS = 256 * 4 * 2.4e9 / 4


def measured_valu(workload_name: str, kernel: str, ms: float):
    """VALU issue of a kernel from the committed rocprofv3 counters
    (SQ_INSTS_VALU per launch) over its live-measured time, against the issue
    peak; None when no summary exists or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"trsv_{workload_name}_traffic.json")
    if not os.path.exists(path) or not ms:
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("per_launch", {}).get(kernel, {})
    if t.get("kernel_sources_hash") != kernel_sources_hash() or "valu_insts" not in k:
        return None
    rate = k["valu_insts"] / (ms * 1e-3)
    return {"insts_per_launch": k["valu_insts"], "achieved": rate, "peak": VALU_PEAK_INSTS,
            "unit": "wave64 VALU instructions/s", "frac": rate / VALU_PEAK_INSTS,
            "source": f"profiles/trsv_{workload_name}_traffic.json (SQ_INSTS_VALU) over this run's time"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(m, budget_s: float = 15.0):
    import oracle
    b = np.ones(m.n)
    solve = oracle.solve_upper if m.meta.get("upper") else oracle.solve
    t0 = time.perf_counter()
    reps = 0
    while True:
        solve(m, b)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    return {"value": reps * m.n / el, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} serial solves of the full matrix ({el:.1f} s), single host thread",
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def parallel_cpu_baseline(workload_name: str, seconds: float = 10.0):
    """The paper's kind of CPU number (Sec. 6.1): the schedule executed on all
    host threads by oracle/executor.c, in a child process so that its OpenMP
    thread placement applies.  None if it fails."""
    import subprocess
    cmd = [sys.executable, "-m", "oracle.executor_bench", "--workload", workload_name, "--seconds", str(seconds)]
    try:
        r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            log(f"parallel executor baseline failed: {r.stderr[-500:]}")
            return None
        d = json.loads(r.stdout.strip().splitlines()[-1])
        d["cpu_model"] = cpu_model()
        return d
    except (subprocess.TimeoutExpired, ValueError, IndexError) as e:
        log(f"parallel executor baseline failed: {e}")
        return None


def schedule_key(core, sup, perm) -> str:
    """SHA-256 of the per-row core, superstep and Sec. 5 order as
    little-endian int32 (the key tests/golden/schedule_keys.json stores for
    the oracle's schedules)."""
    import hashlib
    h = hashlib.sha256()
    for a in (core, sup, perm):
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def golden_schedule_key(name: str):
    path = os.path.join(ROOT, "tests", "golden", "schedule_keys.json")
    try:
        with open(path) as f:
            return json.load(f).get(name)
    except (OSError, ValueError):
        return None


def timed_ms(fn, reps: int, stream) -> float:
    """Mean milliseconds of fn() over reps calls between two events on stream
    (one untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def calibrate_bound(B, stream, reps: int = 20) -> dict:
    """Costs of the persistent kernel for the bound t >= t0 + S t_sync +
    sum_s max_p w(task p of superstep s) t_entry (Sec. 2.3, Eq. (3.1) with
    measured constants): t0 = one launch (64 independent rows), t_entry = one
    stored entry on a lane's serial path (a 2,048-row chain on one core, each
    row reading the previous one on chip), t_sync = one superstep's barrier
    (the same chain as 2,048 one-row supersteps)."""
    import torch
    from paper_2503_05408_amd import gen
    chain = gen.chain(2048)
    b = torch.ones(chain.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with B.Plan(gen.edgeless(64), B.default_opts()) as p0:
        b0 = torch.ones(64, dtype=torch.float64, device="cuda")
        x0 = torch.empty_like(b0)
        t0 = timed_ms(lambda: p0.solve(b0, x0), reps, stream) * 1e3
    zeros = np.zeros(chain.n, dtype=np.int32)
    with B.Plan(chain, B.default_opts(), schedule=(zeros, zeros)) as p1:   # one core, one superstep
        t1 = timed_ms(lambda: p1.solve(b, x), reps, stream) * 1e3
    with B.Plan(chain, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)) as pw:
        S = pw.info()["supersteps"]
        tw = timed_ms(lambda: pw.solve(b, x), reps, stream) * 1e3
        # semi-asynchronous: every row waits for the previous one through memory
        ta = timed_ms(lambda: pw.solve_async(b, x), reps, stream) * 1e3
    with B.Plan(gen.edgeless(64), B.default_opts()) as p0:
        t0a = timed_ms(lambda: p0.solve_async(b0, x0), reps, stream) * 1e3
    # the same chain and launch through the wave-core (record-stream) form
    wave = B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)
    with B.Plan(chain, wave) as pv:
        tv = timed_ms(lambda: pv.solve_async(b, x), reps, stream) * 1e3
    with B.Plan(gen.edgeless(64), wave) as p0:
        t0v = timed_ms(lambda: p0.solve_async(b0, x0), reps, stream) * 1e3
    t_entry = max(0.0, (t1 - t0) / chain.nnz)
    t_sync = max(0.0, (tw - t0) / S - 2 * t_entry)
    hops = {"lane cores": (max(0.0, (ta - t0a) / S), t0a), "wave cores": (max(0.0, (tv - t0v) / S), t0v)}
    t_hop, t0h = min(hops.values())
    return {"t0_us": t0, "t_entry_us": t_entry, "t_sync_us": t_sync, "t0_async_us": t0h, "t_hop_us": t_hop,
            "t_hop_by_form_us": {k: v[0] for k, v in hops.items()},
            "calibration": "edgeless n=64 (t0, t0_async), 2,048-row chain on one core (t_entry), the chain as "
                           "2,048 supersteps in the persistent kernel (t_sync) and in the semi-asynchronous "
                           "forms, lane cores and wave cores (t_hop: a row waiting for its parent through "
                           "memory; the smaller of the two, with that form's launch as t0_async)"}


def third_bound(plan, m, cal: dict) -> dict:
    """The bound of Sec. 2.3 / Eq. (3.1) for a lane-core plan: S superstep
    barriers plus, per superstep, the stored entries of its heaviest task
    walked one after another by one lane."""
    core, sup, _ = plan.schedule()
    w = np.diff(np.asarray(m.row_ptr, dtype=np.int64))
    key = sup.astype(np.int64) * (int(core.max()) + 1 if core.size else 1) + core
    order = np.argsort(key, kind="stable")
    ks = key[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]]) if ks.size else np.zeros(0, np.int64)
    task_w = np.add.reduceat(w[order], starts) if ks.size else np.zeros(0)
    task_s = sup[order][starts]
    S = int(plan.info()["supersteps"])
    crit = np.zeros(max(S, 1))
    np.maximum.at(crit, task_s, task_w)
    W = float(crit.sum())
    us = cal["t0_us"] + S * cal["t_sync_us"] + W * cal["t_entry_us"]
    levels = int(plan.info()["wavefronts"])
    return {"ms": us * 1e-3, "supersteps": S, "critical_entries": int(W),
            "formula": "t0 + S t_sync + (sum over supersteps of the heaviest task's entries) t_entry",
            "async_ms": (cal["t0_async_us"] + levels * cal["t_hop_us"]) * 1e-3, "wavefronts": levels,
            "async_formula": "t0_async + wavefronts t_hop (semi-asynchronous forms: one memory hop per "
                             "level of the DAG)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="er1e7")
    ap.add_argument("--schedule", default="growlocal", choices=["growlocal", "wavefront", "auto"])
    ap.add_argument("--L", type=float, default=50.0)
    ap.add_argument("--alpha0", type=float, default=1.0)
    ap.add_argument("--k", type=int, default=1 << 16)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "analysis", "paper"],
                    help="single: one n=1e7 system (the headline line); batch: 64 systems in one launch; "
                         "serve: Poisson request stream against resident plans; analysis: analysis time, "
                         "supersteps and solve time against the number of scheduling blocks")
    ap.add_argument("--blocks", default="1,2,4,8,16")
    ap.add_argument("--instances", type=int, default=10, help="paper mode: instances per set")
    ap.add_argument("--funnel", default="",
                    help="analysis mode: comma-separated Funnel part-weight caps to measure as well")
    ap.add_argument("--triangle", default="lower", choices=["lower", "upper"],
                    help="upper: backward substitution on the transpose of the workload")
    ap.add_argument("--systems", type=int, default=64)
    ap.add_argument("--batch-forms", default="all", choices=["all", "wave"],
                    help="batch mode: autotune every form and claim size, or run the wavefront-core "
                         "semi-asynchronous launch only")
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the serving run the default line carries")
    ap.add_argument("--no-extras", action="store_true",
                    help="single mode: leave out the 27-point grid, the 64-system batch, the serving run, "
                         "the schedule check and the third bound")
    ap.add_argument("--quantum-us", type=float, default=200.0)
    ap.add_argument("--async-exec", action="store_true",
                    help="serve mode: semi-asynchronous execution (no superstep barriers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solve has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "analysis":
        return bench_analysis(args)
    if args.mode == "paper":
        return bench_paper(args)

    import torch
    import oracle
    from paper_2503_05408_amd import binding as B

    t = time.time()
    m, desc = workload(args.workload)
    upper = args.triangle == "upper"
    if upper:   # backward substitution on the transpose
        from paper_2503_05408_amd import gen
        m = gen.upper_of(m)
        desc = "transpose (upper triangle, backward substitution) of: " + desc
    log(f"workload {m.name}: n={m.n} nnz={m.nnz} generated in {time.time() - t:.1f} s")
    kind = {"wavefront": B.SCHED_WAVEFRONT, "auto": B.SCHED_AUTO}.get(args.schedule, B.SCHED_GROWLOCAL)
    opts = B.default_opts(k=args.k, L=args.L, alpha0=args.alpha0, schedule_kind=kind,
                          triangle=B.UPPER if upper else B.LOWER)
    solve_ref = oracle.solve_upper if upper else oracle.solve
    t = time.time()
    plan = B.Plan(m, opts)
    info = plan.info()
    log(f"plan: S={info['supersteps']} wavefronts={info['wavefronts']} chunks={info['chunks']} "
        f"grid={info['grid_blocks']} analysis {info['analysis_ns'] / 1e9:.1f} s (wall {time.time() - t:.1f} s)")

    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()

    # exactness gate
    want = solve_ref(m, np.ones(m.n))
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

    # the same schedule without the reorder of Sec. 5 (A in its CSR order,
    # one launch per superstep): the locality comparison of Table 7.3
    core, sup, _ = plan.schedule()
    uopts = B.PlanOpts()
    ctypes.memmove(ctypes.byref(uopts), ctypes.byref(opts), ctypes.sizeof(uopts))
    uopts.reorder = 0
    with B.Plan(m, uopts, schedule=(core, sup)) as uplan:
        x.fill_(float("nan"))
        uplan.solve_unordered(b, x)
        torch.cuda.synchronize()
        exact_unordered = oracle.same_bits(x.cpu().numpy(), want)
        uplan.solve_unordered(b, x)
        u0 = torch.cuda.Event(enable_timing=True)
        u1 = torch.cuda.Event(enable_timing=True)
        u0.record(stream)
        for _ in range(args.plain_steps):
            uplan.solve_unordered(b, x)
        u1.record(stream)
        torch.cuda.synchronize()
        ms_unordered = u0.elapsed_time(u1) / args.plain_steps
    del core, sup

    # wavefront cores (a BSP core is a whole wave) on the wavefront schedule
    wopts = B.PlanOpts()
    ctypes.memmove(ctypes.byref(wopts), ctypes.byref(opts), ctypes.sizeof(wopts))
    wopts.core_width = 64
    wopts.schedule_kind = B.SCHED_WAVEFRONT
    wave = {}
    with B.Plan(m, wopts) as wplan:
        for name, fn in (("persistent", wplan.solve), ("async", wplan.solve_async)):
            x.fill_(float("nan"))
            fn(b, x)
            torch.cuda.synchronize()
            ok = wplan.device_status() == 0 and oracle.same_bits(x.cpu().numpy(), want)
            w0 = torch.cuda.Event(enable_timing=True)
            w1 = torch.cuda.Event(enable_timing=True)
            w0.record(stream)
            for _ in range(args.plain_steps):
                fn(b, x)
            w1.record(stream)
            torch.cuda.synchronize()
            wave[name] = {"ms_per_step": w0.elapsed_time(w1) / args.plain_steps, "exact": bool(ok)}

    # semi-asynchronous form: no barriers, per-row readiness
    x.fill_(0.0)
    plan.solve_async(b, x)
    torch.cuda.synchronize()
    exact_async = oracle.same_bits(x.cpu().numpy(), want) and plan.device_status() == 0
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    for _ in range(args.steps):
        plan.solve_async(b, x)
    a1.record(stream)
    torch.cuda.synchronize()
    ms_async = a0.elapsed_time(a1) / args.steps
    if plan.device_status() != 0:
        exact_async = False

    # several right-hand sides per pass (SpTRSM): columns x rows per second
    multi = {}
    for nrhs in (4, 8):
        Bm = torch.ones(m.n, nrhs, dtype=torch.float64, device="cuda")
        Xm = torch.empty_like(Bm)
        plan.solve_multi(Bm, Xm)
        torch.cuda.synchronize()
        ok = plan.device_status() == 0 and all(oracle.same_bits(Xm[:, r].cpu().numpy(), want) for r in (0, nrhs - 1))
        q0 = torch.cuda.Event(enable_timing=True)
        q1 = torch.cuda.Event(enable_timing=True)
        q0.record(stream)
        reps = max(1, args.steps // 4)
        for _ in range(reps):
            plan.solve_multi(Bm, Xm)
        q1.record(stream)
        torch.cuda.synchronize()
        ms_m = q0.elapsed_time(q1) / reps
        multi[str(nrhs)] = {"ms_per_step": ms_m, "exact": bool(ok),
                            "rhs_rows_per_s": (m.n * nrhs / (ms_m * 1e-3)) if ok else 0.0}
        del Bm, Xm

    # plain form with its S launches captured once in a hipGraph and replayed
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.solve_plain(b, x)
    x.fill_(float("nan"))
    graph.replay()
    torch.cuda.synchronize()
    exact_graph = oracle.same_bits(x.cpu().numpy(), want)
    q0 = torch.cuda.Event(enable_timing=True)
    q1 = torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for _ in range(args.plain_steps):
        graph.replay()
    q1.record(stream)
    torch.cuda.synchronize()
    ms_graph = q0.elapsed_time(q1) / args.plain_steps
    del graph

    # the same bytes without the dependencies: one gather-probe pass over the plan
    ones = torch.ones_like(x)
    ysink = torch.zeros_like(x)
    plan.gather_probe(ones, ysink)
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(5):
        plan.gather_probe(ones, ysink)
    g1.record(stream)
    torch.cuda.synchronize()
    gather_ms = g0.elapsed_time(g1) / 5
    del ones, ysink

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
    default_run = args.workload == "er1e7" and args.schedule == "growlocal" and not upper
    traffic = measured_traffic(args.workload if default_run else
                               f"{args.workload}_{args.schedule}" + ("_upper" if upper else ""),
                               "trsv_persistent")
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
        "exact": bool(exact and exact_plain and exact_graph),
        "nnz_per_s": m.nnz / (ms * 1e-3),
        "gflops": (2 * m.nnz - m.n) / (ms * 1e-3) / 1e9,
        "plain": {"value": rows_s_plain, "ms_per_step": ms_plain, "launches_per_step": info["supersteps"],
                  "graph_ms_per_step": ms_graph},
        "speedup_vs_plain": (ms_plain / ms) if ms > 0 else None,
        "wave_cores_wavefront": wave,
        "unordered": {"ms_per_step": ms_unordered, "exact": bool(exact_unordered),
                      "reorder_speedup": (ms_unordered / ms_plain) if ms_plain > 0 else None},
        "multi_rhs": multi,
        "async": {"ms_per_step": ms_async, "exact": bool(exact_async),
                  "value": (m.n / (ms_async * 1e-3)) if exact_async else 0.0},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "iqr": float(np.percentile(per, 75) - np.percentile(per, 25))},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "trsv_persistent", "alg_bytes_per_launch": alg, "kernel_ms": kern_ms,
            "copy_probe_GBs": copy_gbs,
            "gather_floor_ms": gather_ms,
            "frac_of_gather_floor": gather_ms / kern_ms if kern_ms > 0 else None,
            "traffic_GBs": (traffic / (kern_ms * 1e-3) / 1e9) if traffic else None,
            "valu": measured_valu("er1e7", "trsv_persistent", kern_ms),
        },
    }
    prop = torch.cuda.get_device_properties(0)
    out["device"] = {"name": prop.name, "arch": getattr(prop, "gcnArchName", ""),
                     "compute_units": prop.multi_processor_count,
                     "memory_GB": round(prop.total_memory / 1e9, 1)}
    if default_run and not args.no_extras:
        # the schedule against the oracle's (Alg. 3.1 + Sec. 5) at this size
        core, sup, perm = plan.schedule()
        gold = golden_schedule_key("bench_er_n1e7")
        key = schedule_key(core, sup, perm)
        out["schedule_vs_oracle"] = {"key": key[:16], "golden": (gold or {}).get("key", "")[:16],
                                     "equal": bool(gold and gold.get("key") == key),
                                     "source": "tests/golden/schedule_keys.json (written from the oracle only)"}
        del core, sup, perm
        cal = calibrate_bound(B, stream)
        out["third_bound_calibration"] = cal
        out["third_bound"] = third_bound(plan, m, cal)
        out["third_bound"]["frac"] = out["third_bound"]["ms"] / ms                 # of the persistent solve
        out["third_bound"]["async_frac"] = out["third_bound"]["async_ms"] / ms_async
    plan.close()
    if default_run and not args.no_extras:
        side = torch.cuda.Stream()   # graph capture needs a stream other than the default one
        log("C2(ii): 27-point grid ...")
        out["c2_st27"] = extra_st27(B, stream, cal, reps=10)
        log(f"  {out['c2_st27']['form']} {out['c2_st27']['ms_per_step']:.3f} ms")
        log("C3: 64-system batch ...")
        out["c3_batch"] = extra_c3(B, side, cal, reps=10)
        log(f"  {out['c3_batch']['ms_per_step']:.3f} ms")
        log("C5: serving ...")
        out["c5_serve"] = serve_run(args.pool, args.rate, args.serve_seconds, args.quantum_us, args.async_exec)
        log(f"  p50 {out['c5_serve']['latency_ms']['p50']} ms p99 {out['c5_serve']['latency_ms']['p99']} ms")
        # the same stream through the other execution form of the server
        out["c5_serve_other_form"] = serve_run(args.pool, args.rate, args.serve_seconds, args.quantum_us,
                                               not args.async_exec)
        log(f"  ({out['c5_serve_other_form']['form']}) p50 {out['c5_serve_other_form']['latency_ms']['p50']} ms "
            f"p99 {out['c5_serve_other_form']['latency_ms']['p99']} ms")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(m)
        if default_run:
            log("cpu baseline (parallel executor of the schedule, all host threads) ...")
            par = parallel_cpu_baseline(args.workload)
            if par:
                par["speedup_over_serial"] = par["value"] / out["cpu_baseline"]["value"]
                out["cpu_baseline"]["parallel_executor"] = par
    print(json.dumps(out), flush=True)


def bench_analysis(args):
    """Block-parallel scheduling (Sec. 3.1) on one workload: for each block
    count, the plan's analysis time, supersteps and persistent solve time,
    and the solves after which the GrowLocal plan repays its extra analysis
    time over the wavefront plan (Table 7.6/7.7 analogue)."""
    import torch
    import oracle
    from paper_2503_05408_amd import binding as B
    m, desc = workload(args.workload)
    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    want = oracle.solve(m, np.ones(m.n))
    stream = torch.cuda.current_stream()

    def measure(opts):
        t0 = time.perf_counter()
        plan = B.Plan(m, opts)
        wall = time.perf_counter() - t0
        info = plan.info()
        x = plan.solve(b)
        torch.cuda.synchronize()
        exact = oracle.same_bits(x.cpu().numpy(), want)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            plan.solve(b, x)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.close()
        return {"analysis_s": info["analysis_ns"] / 1e9, "plan_wall_s": wall, "supersteps": info["supersteps"],
                "solve_ms": e0.elapsed_time(e1) / args.steps, "exact": bool(exact)}

    t0 = time.perf_counter()
    oracle.solve(m, np.ones(m.n))
    serial_s = time.perf_counter() - t0          # one serial solve on one host core
    wf = measure(B.default_opts(schedule_kind=B.SCHED_WAVEFRONT))
    log(f"wavefront: {wf}; serial CPU solve {serial_s:.3f} s")
    rows = []
    for nb in [int(v) for v in args.blocks.split(",")]:
        r = measure(B.default_opts(k=args.k, L=args.L, alpha0=args.alpha0, blocks=nb))
        gain_ms = wf["solve_ms"] - r["solve_ms"]
        r["blocks"] = nb
        r["repay_solves_vs_wavefront"] = ((r["analysis_s"] - wf["analysis_s"]) * 1e3 / gain_ms
                                          if gain_ms > 0 else None)
        # Table 7.6's threshold: scheduling time over the time one solve saves
        # against the serial solve
        r["repay_solves_vs_cpu_serial"] = r["analysis_s"] / (serial_s - r["solve_ms"] * 1e-3)
        log(f"blocks={nb}: {r}")
        rows.append(r)
    frows = []
    for cap in [int(v) for v in args.funnel.split(",") if v]:
        r = measure(B.default_opts(k=args.k, L=args.L, alpha0=args.alpha0, funnel_max_weight=cap))
        r["funnel_max_weight"] = cap
        log(f"funnel cap={cap}: {r}")
        frows.append(r)
    print(json.dumps({"mode": "analysis", "workload": desc, "n": m.n, "nnz": m.nnz, "funnel": frows,
                      "schedule": f"growlocal k={args.k} L={args.L:g} alpha0={args.alpha0:g}",
                      "host_threads": os.cpu_count(), "serial_cpu_solve_s": serial_s, "wavefront": wf,
                      "blocks": rows}), flush=True)


def bench_paper(args):
    """The paper's synthetic sets at paper size (ER p in {1e-4, 5e-4, 2e-3} and
    NB (p, B) in {(0.14, 10), (0.05, 20), (0.03, 42)}, n = 1e5, ten instances
    each): per set, the geometric mean over instances of the speed-up over one
    serial solve on one host core (the kind of number of Table 7.1) for each
    schedule and execution form, and the mean ratio wavefronts / supersteps
    (Table 7.2).  Every timed result is checked against the oracle bit for
    bit."""
    import torch
    import oracle
    from paper_2503_05408_amd import binding as B
    from paper_2503_05408_amd import gen
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    sets = [("ER", p, None) for p in gen.ER_PROBS] + [("NB", p, Bw) for p, Bw in gen.NB_PAIRS]
    o_gl, o_wf, o_auto = B.gpu_opts(), B.default_opts(schedule_kind=B.SCHED_WAVEFRONT), \
        B.gpu_opts(schedule_kind=B.SCHED_AUTO)
    o_auto_a = B.gpu_opts(schedule_kind=B.SCHED_AUTO, exec_hint=1)
    o_wave = B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)
    forms = {"GL persistent": (o_gl, "solve"), "GL async": (o_gl, "solve_async"),
             "wavefront persistent": (o_wf, "solve"), "wavefront async": (o_wf, "solve_async"),
             "AUTO persistent": (o_auto, "solve"), "AUTO async": (o_auto_a, "solve_async"),
             "wavefront wave-core persistent": (o_wave, "solve"),
             "wavefront wave-core async": (o_wave, "solve_async")}
    report = []
    for fam, p, Bw in sets:
        logs = {f: [] for f in forms}
        ratios, all_exact = [], True
        kept, serial_total = [], 0.0   # (matrix, wavefront plan, AUTO plan, want) for the batched launches
        for i in range(args.instances):
            m = (gen.erdos_renyi_paper(100_000, p, gen.SEED_BASE + i) if fam == "ER"
                 else gen.narrow_band(100_000, p, Bw, gen.SEED_BASE + 10 + i))
            bh = np.ones(m.n)
            t0 = time.perf_counter()
            want = oracle.solve(m, bh)
            serial = time.perf_counter() - t0
            serial_total += serial
            b = torch.ones(m.n, dtype=torch.float64, device="cuda")
            x = torch.empty_like(b)
            plans = {}
            for f, (o, meth) in forms.items():
                key = id(o)
                if key not in plans:
                    plans[key] = B.Plan(m, o)
                plan = plans[key]
                t = timed(lambda: getattr(plan, meth)(b, x), args.steps)
                ok = plan.device_status() == 0 and oracle.same_bits(x.cpu().numpy(), want)
                all_exact &= ok
                logs[f].append(serial / t)
                if f == "GL persistent":
                    inf = plan.info()
                    ratios.append(inf["wavefronts"] / inf["supersteps"])
            kept.append((m, plans.pop(id(o_auto_a)), plans.pop(id(o_auto)), want, plans.pop(id(o_wave))))
            for plan in plans.values():
                plan.close()
        # every instance of the set in one launch: throughput against the serial solves one after another
        batched = {}
        bs = [torch.ones(k[0].n, dtype=torch.float64, device="cuda") for k in kept]
        xs = [torch.empty_like(v) for v in bs]
        for label, idx, async_exec in (("AUTO async batch", 1, True), ("AUTO BSP batch", 2, False),
                                       ("wavefront wave-core async batch", 4, True)):
            with B.Batch([k[idx] for k in kept], per_claim=2, use_graph=False, async_exec=async_exec) as bt:
                t = timed(lambda: bt.solve(bs, xs), args.steps)
                ok = bt.status() == 0 and all(oracle.same_bits(x.cpu().numpy(), k[3]) for x, k in zip(xs, kept))
            all_exact &= ok
            batched[label] = serial_total / t
        for k in kept:
            k[1].close()
            k[2].close()
            k[4].close()
        row = {"set": f"{fam} p={p}" + (f" B={Bw:g}" if Bw else ""), "instances": args.instances,
               "exact": bool(all_exact), "wavefronts_per_superstep_GL": float(np.mean(ratios)),
               "geomean_speedup_vs_serial": {f: float(np.exp(np.mean(np.log(v)))) for f, v in logs.items()},
               "batched_speedup_vs_serial_sum": batched}
        log(json.dumps(row))
        report.append(row)
    print(json.dumps({"mode": "paper", "n": 100_000, "serial": "oracle, one host core, one solve",
                      "sets": report}), flush=True)


def auto_plan(m, async_exec: bool = False):
    """AUTO schedule, predicted for the execution form that will run it."""
    from paper_2503_05408_amd import binding as B
    return B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO, exec_hint=1 if async_exec else 0))


def bench_batch(args):
    """64 independent systems (n = 10^U[3,6], ER/NB/2-D/3-D mix) in one
    hipGraph-replayed persistent launch, against 64 sequential plain solves."""
    import torch
    import oracle
    from paper_2503_05408_amd import binding as B
    from paper_2503_05408_amd import gen

    t = time.time()
    ms = gen.batch_mix(args.systems)
    log(f"batch: {len(ms)} systems, {sum(m.n for m in ms)} rows, generated in {time.time() - t:.1f} s")
    t = time.time()
    plans = [auto_plan(m) for m in ms]
    plans_async = [auto_plan(m, async_exec=True) for m in ms]
    plans_wave = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) for m in ms]
    log(f"plans in {time.time() - t:.1f} s; supersteps total {sum(p.info()['supersteps'] for p in plans)}, "
        f"max {max(p.info()['supersteps'] for p in plans)}; async-predicted plans: max supersteps "
        f"{max(p.info()['supersteps'] for p in plans_async)}")
    stream = torch.cuda.Stream()
    bd = [torch.ones(m.n, dtype=torch.float64, device="cuda") for m in ms]
    xd = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
    from paper_2503_05408_amd import tuning
    if args.batch_forms == "wave":
        # the semi-asynchronous launch on wavefront cores only (e.g. for profiling)
        with torch.cuda.stream(stream):
            bt = B.Batch(plans_wave, per_claim=1, use_graph=True, async_exec=True)
            ms_w = timed_ms(lambda: bt.solve(bd, xd, stream), args.steps, stream)
        per_claim, form = 1, "wave"
        timings = {"wave_claim1_ms": ms_w}
        ms_b = ms_w
    else:
        # execution form and claim size picked by the autotuner (measured)
        with torch.cuda.stream(stream):
            bt, entry = tuning.best_batch(plans, bd, xd, plans_async=plans_async, plans_wave=plans_wave,
                                          claims=(1, 2, 4, 8), reps=args.steps, stream=stream)
        per_claim, form = entry["per_claim"], entry["form"]
        timings = {f"{k.split('/')[0]}_claim{k.split('/')[1]}_ms": v for k, v in entry["ms"].items()}
        ms_b = timings[f"{form}_claim{per_claim}_ms"]
    log(f"autotuned: {form} per_claim={per_claim} {ms_b:.3f} ms; {timings}")
    for x in xd:
        x.fill_(float("nan"))
    with torch.cuda.stream(stream):
        bt.solve(bd, xd, stream)
        stream.synchronize()
    exact = bt.status() == 0 and all(oracle.same_bits(x.cpu().numpy(), oracle.solve(m, np.ones(m.n)))
                                     for m, x in zip(ms, xd))

    def seq(fn):
        with torch.cuda.stream(stream):
            for p, b, x in zip(plans, bd, xd):
                fn(p)(b, x, stream)
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            reps = max(1, args.plain_steps // 5)
            for _ in range(reps):
                for p, b, x in zip(plans, bd, xd):
                    fn(p)(b, x, stream)
            e1.record(stream)
            stream.synchronize()
        return e0.elapsed_time(e1) / reps

    # (--plain-steps 0 leaves out the sequential comparisons, e.g. under a counter profiler)
    ms_plain = seq(lambda p: p.solve_plain) if args.plain_steps > 0 else None
    ms_pers = seq(lambda p: p.solve) if args.plain_steps > 0 else None
    rows = sum(m.n for m in ms)
    alg = sum(algorithmic_bytes(m.n, m.nnz) for m in ms)
    achieved = alg / (ms_b * 1e-3) / 1e9
    out = {
        "metric": "reduced elements/sec (exact) at 1 MI355X vs plain launch; p50/p99 latency",
        "value": rows / (ms_b * 1e-3) if exact else 0.0, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(ms)} independent systems, n = floor(10^U[3,6]), ER/NB/2-D/3-D mix, "
                               "one hipGraph-replayed persistent launch",
                   "rows": rows, "nnz": sum(m.nnz for m in ms), "per_claim": per_claim, "form": form,
                   "schedule": ("wavefront, wavefront cores" if form == "wave"
                                else "auto (GrowLocal k=65536 L=50 alpha0=1, or wavefront)")},
        "timings": timings,
        "exact": bool(exact),
        "plain_sequential_ms": ms_plain, "persistent_sequential_ms": ms_pers,
        "speedup_vs_plain": (ms_plain / ms_b) if ms_plain else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": {"async": "trsv_batched_async", "wave": "trsv_stream_async"}.get(form, "trsv_batched"),
                     "alg_bytes_per_launch": alg},
    }
    bt.close()
    print(json.dumps(out), flush=True)


def serve_run(pool: int, rate: float, seconds: float, quantum_us: float, async_exec: bool, nb: int = 4) -> dict:
    """Poisson request stream (rate, seconds) against a pool of resident plans
    (n = floor(10^U[0,6])).  Each request solves A x = b for one of `nb`
    seeded right-hand sides of its matrix into a fresh x; every completed x is
    compared bit for bit with the oracle's solution on the device, and only
    the rows of matching requests count.  Latency runs from the scheduled
    arrival to the completion seen by the host."""
    import torch
    from paper_2503_05408_amd import binding as B
    from paper_2503_05408_amd import gen
    import oracle

    t = time.time()
    ms = gen.batch_mix(pool, seed=gen.SEED_BASE + 1000, lo_exp=0.0, hi_exp=6.0)
    plans = [auto_plan(m) for m in ms]
    bs, want = [], []
    for i, m in enumerate(ms):
        bh = [gen.rhs_uniform(m.n, gen.SEED_BASE + 3000 + nb * i + j) for j in range(nb)]
        bs.append([torch.from_numpy(v).cuda() for v in bh])
        want.append([torch.from_numpy(oracle.solve(m, v)).cuda().view(torch.int64) for v in bh])
    torch.cuda.synchronize()
    log(f"serve: pool of {len(ms)} plans ({sum(m.n for m in ms)} rows, {nb} right-hand sides each) "
        f"ready in {time.time() - t:.1f} s")
    rng = np.random.default_rng(gen.SEED_BASE + 2000)
    nreq = int(rate * seconds * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, size=nreq)
    which = rng.integers(0, len(ms), size=nreq)
    rhs = rng.integers(0, nb, size=nreq)
    lat, rows_all, flags = [], [], []
    backlog = []
    inflight = {}
    with B.Server(quantum_us=quantum_us, max_slots=512, budget_bytes=8 << 30, async_exec=int(async_exec)) as sv:
        t0 = B.clock_ns()
        arrival = t0 + np.cumsum(gaps) * 1e9
        end = t0 + seconds * 1e9
        nxt = 0
        last_log = t0
        while True:
            now = B.clock_ns()
            while nxt < nreq and arrival[nxt] <= now and arrival[nxt] <= end:
                backlog.append(nxt)
                nxt += 1
            while backlog:
                r = backlog[0]
                i = int(which[r])
                x = torch.empty(ms[i].n, dtype=torch.float64, device="cuda")
                tk = sv.submit(plans[i], bs[i][int(rhs[r])], x)
                if tk is None:
                    break
                inflight[tk] = (r, i, x)
                backlog.pop(0)
            for tk, done_ns in sv.poll():
                r, i, x = inflight.pop(tk)
                lat.append((done_ns - arrival[r]) * 1e-6)
                rows_all.append(ms[i].n)
                # compared on the device without a host sync: one flag per request
                flags.append(torch.ne(x.view(torch.int64), want[i][int(rhs[r])]).any())
            if now >= end and not inflight and not backlog:
                break
            if now - last_log > 10e9:
                log(f"serve: t={(now - t0) * 1e-9:.0f}s completed={len(lat)} inflight={len(inflight)} "
                    f"backlog={len(backlog)}")
                last_log = now
            time.sleep(0.0001)
        elapsed = (B.clock_ns() - t0) * 1e-9
        st = sv.stats()
    bad = torch.stack(flags).cpu().numpy() if flags else np.zeros(0, dtype=bool)
    rows_all = np.asarray(rows_all, dtype=np.int64)
    rows_ok = int(rows_all[~bad].sum()) if rows_all.size else 0
    lat = np.array(lat)
    for p in plans:
        p.close()
    return {
        "value": rows_ok / elapsed, "unit": "rows/s",
        "workload": f"Poisson {rate:g} requests/s for {seconds:g} s, pool of {len(ms)} resident plans "
                    f"n = floor(10^U[0,6]) (ER/NB/2-D/3-D mix), {nb} seeded right-hand sides per matrix",
        "form": "async" if async_exec else "bsp", "quantum_us": quantum_us,
        "latency_ms": {"p50": float(np.percentile(lat, 50)) if lat.size else None,
                       "p99": float(np.percentile(lat, 99)) if lat.size else None,
                       "max": float(lat.max()) if lat.size else None},
        "requests": int(lat.size), "checked_exact": int(lat.size), "mismatches": int(bad.sum()),
        "exact": bool(lat.size and not bad.any()), "rows_checked": rows_ok,
        "launches": st["launches"], "elapsed_s": elapsed,
    }


def bench_serve(args):
    """The serving benchmark on its own (see serve_run)."""
    r = serve_run(args.pool, args.rate, args.seconds, args.quantum_us, args.async_exec)
    out = {
        "metric": "reduced elements/sec (exact) at 1 MI355X vs plain launch; p50/p99 latency",
        "value": r["value"], "unit": "rows/s", "n_gpus": 1,
        "steps": r["requests"], "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r["workload"], "quantum_us": r["quantum_us"], "form": r["form"]},
    }
    out.update({k: v for k, v in r.items() if k not in ("value", "unit", "workload", "form", "quantum_us")})
    print(json.dumps(out), flush=True)


def run_forms(plan, forms, b, x, want, reps, stream):
    """ms per solve and bit-exactness for each named solve method of plan."""
    import torch
    import oracle
    out = {}
    for name in forms:
        fn = getattr(plan, name)
        x.fill_(float("nan"))
        fn(b, x)
        torch.cuda.synchronize()
        ok = plan.device_status() == 0 and oracle.same_bits(x.cpu().numpy(), want)
        ms = timed_ms(lambda: fn(b, x), reps, stream)
        ok = ok and plan.device_status() == 0
        out[name] = {"ms": ms, "exact": bool(ok)}
    return out


def extra_st27(B, stream, cal, reps: int) -> dict:
    """C2(ii): the 3-D 27-point 216^3 grid, one system, every form."""
    import torch
    import oracle
    from paper_2503_05408_amd import gen
    t = time.time()
    m = gen.stencil_3d27(216)
    want = oracle.solve(m, np.ones(m.n))
    log(f"st27: generated and solved on the host in {time.time() - t:.1f} s")
    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    res = {}
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) as lp:
        inf = lp.info()
        for k, v in run_forms(lp, ("solve", "solve_async", "solve_plain"), b, x, want, reps, stream).items():
            res["lane " + k] = v
        bound = third_bound(lp, m, cal)
        sched = "wavefront" if inf["schedule_kind"] == B.SCHED_WAVEFRONT else "growlocal"
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) as wp:
        for k, v in run_forms(wp, ("solve_async",), b, x, want, reps, stream).items():
            res["wave-core " + k] = v
    out = summarize(m, "3-D 27-point Laplacian lower triangle 216^3 (n=10,077,696), b = ones",
                    res, "lane solve_plain", bound, f"AUTO -> {sched} (k=65536 L=50 alpha0=1); wave cores: wavefront",
                    inf["supersteps"])
    kern = {"lane solve": "trsv_persistent", "lane solve_async": "trsv_async",
            "wave-core solve_async": "trsv_stream_async"}.get(out["form"])
    traffic = measured_traffic("st27", kern) if kern else None
    out["roofline"].update(kernel=kern, traffic=traffic,
                           traffic_GBs=(traffic / (out["ms_per_step"] * 1e-3) / 1e9) if traffic else None,
                           valu=measured_valu("st27", kern, out["ms_per_step"]) if kern else None)
    return out


def summarize(m, desc, res, plain_key, bound, schedule, S, pers_key="lane solve"):
    exact = all(v["exact"] for v in res.values())
    ok = {k: v["ms"] for k, v in res.items() if v["exact"]}
    best = min(ok, key=ok.get) if ok else None
    ms = ok[best] if best else None
    alg = algorithmic_bytes(m.n, m.nnz)
    return {
        "workload": desc, "n": int(m.n), "nnz": int(m.nnz), "schedule": schedule, "supersteps": int(S),
        "exact": bool(exact), "form": best, "ms_per_step": ms,
        "value": (m.n / (ms * 1e-3)) if ms else 0.0, "unit": "rows/s",
        "forms_ms": {k: v["ms"] for k, v in res.items()},
        "speedup_vs_plain": (res[plain_key]["ms"] / ms) if ms and res.get(plain_key) else None,
        "roofline": {"bound": "hbm", "alg_bytes_per_solve": alg, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "achieved": (alg / (ms * 1e-3) / 1e9) if ms else None,
                     "frac": (alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if ms else None,
                     "note": "12 nnz + 16 n bytes over the whole solve time"},
        "third_bound": dict(bound,
                            frac=(bound["ms"] / res[pers_key]["ms"]) if res.get(pers_key) else None,
                            async_frac=(bound["async_ms"] / ms) if ms else None,
                            note="frac: BSP bound over the persistent solve (" + pers_key + "); async_frac: "
                                 "semi-asynchronous bound over the fastest form"),
    }


def extra_c3(B, stream, cal, reps: int) -> dict:
    """C3: 64 independent systems in one hipGraph-replayed launch against 64
    plain solves one after another."""
    import torch
    import oracle
    from paper_2503_05408_amd import gen
    t = time.time()
    ms = gen.batch_mix(64)
    want = [oracle.solve(m, np.ones(m.n)) for m in ms]
    lane = [auto_plan(m) for m in ms]
    wave = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) for m in ms]
    log(f"c3: 64 systems, {sum(m.n for m in ms)} rows, plans in {time.time() - t:.1f} s")
    bd = [torch.ones(m.n, dtype=torch.float64, device="cuda") for m in ms]
    xd = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
    try:
        with torch.cuda.stream(stream):
            with B.Batch(wave, per_claim=1, use_graph=True, async_exec=True) as bt:
                bt.solve(bd, xd, stream)
                stream.synchronize()
                exact = bt.status() == 0 and all(oracle.same_bits(x.cpu().numpy(), w) for x, w in zip(xd, want))
                ms_b = timed_ms(lambda: bt.solve(bd, xd, stream), reps, stream)
                exact = exact and bt.status() == 0

            def plain_all():
                for p, b, x in zip(lane, bd, xd):
                    p.solve_plain(b, x, stream)
            for x in xd:
                x.fill_(float("nan"))
            plain_all()
            stream.synchronize()
            exact_plain = all(oracle.same_bits(x.cpu().numpy(), w) for x, w in zip(xd, want))
            ms_plain = timed_ms(plain_all, max(1, reps // 5), stream)
        bounds = [third_bound(p, m, cal) for p, m in zip(lane, ms)]
    finally:
        for p in lane + wave:
            p.close()
    rows, nnz = sum(m.n for m in ms), sum(m.nnz for m in ms)
    alg = sum(algorithmic_bytes(m.n, m.nnz) for m in ms)
    worst = max(bounds, key=lambda d: d["ms"])
    worst_a = max(bounds, key=lambda d: d["async_ms"])
    return {
        "workload": "64 independent systems, n = floor(10^U[3,6]), ER/NB/2-D/3-D mix, b = ones; "
                    "one hipGraph replay: b copied into one vector, one semi-asynchronous record-stream "
                    "launch over the batch's global task order on wavefront cores, x copied back",
        "rows": rows, "nnz": nnz, "exact": bool(exact and exact_plain), "ms_per_step": ms_b,
        "value": rows / (ms_b * 1e-3) if exact else 0.0, "unit": "rows/s",
        "plain_sequential_ms": ms_plain, "speedup_vs_plain": ms_plain / ms_b,
        "roofline": {"bound": "hbm", "alg_bytes_per_solve": alg, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "achieved": alg / (ms_b * 1e-3) / 1e9, "frac": alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "kernel": "trsv_stream_async",
                     "traffic": measured_traffic("c3", "trsv_stream_async"),
                     "valu": measured_valu("c3", "trsv_stream_async", ms_b)},
        "third_bound": {"ms": worst["ms"], "supersteps": worst["supersteps"],
                        "critical_entries": worst["critical_entries"],
                        "formula": "the largest single-system BSP bound (lane-core AUTO plans) of the 64: "
                                   "t0 + S t_sync + (heaviest task entries per superstep) t_entry",
                        "async_ms": worst_a["async_ms"], "wavefronts": worst_a["wavefronts"],
                        "async_frac": worst_a["async_ms"] / ms_b,
                        "async_formula": "the largest single-system semi-asynchronous bound of the 64: "
                                         "t0_async + wavefronts t_hop"},
    }


if __name__ == "__main__":
    main()
