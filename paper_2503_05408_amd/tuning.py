"""Autotune cache for the execution form of a plan.

A plan solves the same system in three forms that give the same bits
(persistent BSP kernel, one launch per superstep, semi-asynchronous); which
is fastest depends on the matrix, its schedule and the device.
``Plan.tune`` measures them (``gltrsv_plan_tune``); this module keeps the
results in a JSON file keyed by what they depend on, so later processes set
the preferred form (``gltrsv_plan_set_exec``) without measuring again.
"""
from __future__ import annotations

import json
import os

from . import binding as B


def tuning_key(plan) -> str:
    """The sparsity pattern (hash), the triangle, the schedule's shape
    (supersteps, tasks, kind) and the device (name, architecture)."""
    import torch
    inf = plan.info()
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", "")
    tri = "upper" if plan.opts.triangle == B.UPPER else "lower"
    return (f"{inf['pattern_key']:016x}/{tri}/S{inf['supersteps']}-T{inf['tasks']}-K{inf['schedule_kind']}/"
            f"{dev.name}/{arch}")


def load_table(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        table = json.load(f)
    if not isinstance(table, dict):
        raise ValueError(f"{path}: not a tuning table")
    return table


def store_table(path: str, table: dict) -> None:
    """Writes the table atomically (a reader never sees a partial file)."""
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_cached(plan, path: str, reps: int = 5) -> str:
    """Sets the plan's preferred form from the table in `path`, measuring
    and storing it first when the table has no entry for the plan.  Returns
    the form's name."""
    key = tuning_key(plan)
    table = load_table(path)
    names = {v: k for k, v in B.EXEC_NAMES.items()}
    hit = table.get(key)
    if isinstance(hit, dict) and hit.get("form") in names:
        plan.set_exec(names[hit["form"]])
        return hit["form"]
    res = plan.tune(reps=reps)
    table = load_table(path)   # another process may have added entries meanwhile
    table[key] = res
    store_table(path, table)
    return res["form"]


SCHEDULES = {B.SCHED_GROWLOCAL: "growlocal", B.SCHED_WAVEFRONT: "wavefront"}


def matrix_key(m, opts) -> str:
    """Identifies a plan before it exists: a hash of the sparsity pattern,
    the triangle, every schedule parameter except the kind, and the device."""
    import hashlib

    import numpy as np
    import torch
    h = hashlib.blake2b(digest_size=12)
    h.update(np.int64(m.n).tobytes())
    h.update(np.ascontiguousarray(m.row_ptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(m.col, dtype=np.int32).tobytes())
    tri = "upper" if opts.triangle == B.UPPER else "lower"
    sig = (f"k{opts.k}-L{opts.L:g}-a{opts.alpha0:g}-g{opts.growth:g}-t{opts.accept:g}-b{opts.blocks}"
           f"-f{opts.funnel_max_weight}")
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{h.hexdigest()}/{tri}/{sig}/{dev.name}/{getattr(dev, 'gcnArchName', '')}"


def best_plan(m, opts=None, path: str | None = None, reps: int = 5, core_widths=(1,), params=None,
              local: bool = False):
    """A plan for m with the measured-fastest schedule, core width, schedule
    parameters and execution form for gltrsv_solve_auto.

    Candidates: for every core width in `core_widths` (1 = a core is a
    lane, 64 = a core is a wavefront), the wavefront schedule and GrowLocal
    at every (k, L) pair in `params` (default: the options' own; the
    paper's L is architecture-dependent, Sec. 3 footnote and Appendix C, and
    its Table 7.5 varies k); with `local`, also the one-workgroup form
    (exec_hint 2) on GrowLocal with k = 64, L = 5 and on the dealt wavefront
    schedule.  Each candidate plan is timed in all its forms
    (``Plan.tune``).  With `path`, the choice is read from / stored in the
    JSON table there, so a later process builds only the chosen plan.
    Returns (plan, entry) with entry = {"label" (the candidate), "schedule",
    "core_width", "k", "L", "exec_hint", "form", "us" (per candidate and
    form)}."""
    import ctypes
    base = opts if opts is not None else B.gpu_opts()
    params = [(int(k), float(L)) for k, L in (params or [(base.k, base.L)])]

    def variant(kind, width, k=None, L=None, hint=None):
        o = B.PlanOpts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(base), ctypes.sizeof(o))
        o.schedule_kind = kind
        o.core_width = width
        if k is not None:
            o.k = k
        if L is not None:
            o.L = L
        if hint is not None:
            o.exec_hint = hint
        return o

    cands = []   # (label, schedule name, opts)
    for width in core_widths:
        cands.append((f"wavefront/w{width}", "wavefront", width, None, None, base.exec_hint,
                      variant(B.SCHED_WAVEFRONT, width)))
        for k, L in params:
            cands.append((f"growlocal-k{k}-L{L:g}/w{width}", "growlocal", width, k, L, base.exec_hint,
                          variant(B.SCHED_GROWLOCAL, width, k, L)))
    if local:
        cands.append(("local-growlocal-k64-L5/w1", "growlocal", 1, 64, 5.0, 2,
                      variant(B.SCHED_GROWLOCAL, 1, 64, 5.0, 2)))
        cands.append(("local-wavefront/w1", "wavefront", 1, None, None, 2, variant(B.SCHED_WAVEFRONT, 1, hint=2)))
    names = {v: k for k, v in SCHEDULES.items()}
    forms = {v: k for k, v in B.EXEC_NAMES.items()}
    sig = "/".join(c[0] for c in cands)
    key = f"{matrix_key(m, base)}/{sig}" if path else None
    if path:
        hit = load_table(path).get(key)
        if isinstance(hit, dict) and hit.get("schedule") in names and hit.get("form") in forms:
            plan = B.Plan(m, variant(names[hit["schedule"]], int(hit.get("core_width", 1)), hit.get("k"),
                                     hit.get("L"), hit.get("exec_hint")))
            plan.set_exec(forms[hit["form"]])
            return plan, hit
    best, best_us, times = None, None, {}
    for label, sname, width, k, L, hint, o in cands:
        plan = B.Plan(m, o)
        res = plan.tune(reps=reps)
        usable = res["us"]
        for f, us in usable.items():
            times[f"{label}/{f}"] = us
        form = min(usable, key=usable.get)
        if best_us is None or usable[form] < best_us:
            if best is not None:
                best[0].close()
            best, best_us = (plan, label, sname, width, k, L, hint, form), usable[form]
        else:
            plan.close()
    plan, label, sname, width, k, L, hint, form = best
    plan.set_exec(forms[form])
    entry = {"label": label, "schedule": sname, "core_width": width, "k": k, "L": L, "exec_hint": hint,
             "form": form, "us": times}
    if path:
        table = load_table(path)
        table[key] = entry
        store_table(path, table)
    return plan, entry


def _batch_key(plans, plans_async) -> str:
    import hashlib

    import torch
    h = hashlib.blake2b(digest_size=12)
    for group in (plans, plans_async or []):
        for p in group:
            h.update(tuning_key(p).encode())
        h.update(b"|")
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"batch/{h.hexdigest()}/{dev.name}/{getattr(dev, 'gcnArchName', '')}"


def best_batch(plans, b, x, plans_async=None, claims=(1, 2, 4, 8), reps: int = 3, path: str | None = None,
               stream=None, plans_wave=None):
    """The batched launch (gltrsv_batch_*) with the measured-fastest chunk
    claim size and execution form for this set of systems: BSP on `plans`,
    and, when `plans_async` (the same systems, e.g. planned for
    semi-asynchronous execution) is given, semi-asynchronous on those, and
    when `plans_wave` (the same systems with core width 64) is given,
    semi-asynchronous on wavefront cores ("wave").  b and
    x: lists of device tensors per system, not aliasing each other; x ends
    holding the solutions.  With `path` the choice is read from / stored in
    the JSON table there.  Returns (batch, entry) with entry = {"form",
    "per_claim", "ms"}; the caller closes the batch."""
    import torch
    stream = stream or torch.cuda.current_stream()
    forms = [("bsp", plans)] + ([("async", plans_async)] if plans_async is not None else []) + \
        ([("wave", plans_wave)] if plans_wave is not None else [])
    key = _batch_key(plans, (plans_async or []) + (plans_wave or [])) if path else None
    if path:
        hit = load_table(path).get(key)
        if isinstance(hit, dict) and hit.get("form") in dict(forms) and int(hit.get("per_claim", 0)) >= 1:
            bt = B.Batch(dict(forms)[hit["form"]], per_claim=int(hit["per_claim"]), use_graph=True,
                         async_exec=hit["form"] != "bsp")
            return bt, hit
    best, times = None, {}
    for form, ps in forms:
        for pc in (claims if form != "wave" else (1,)):   # wave batches run a static task order
            bt = B.Batch(ps, per_claim=pc, use_graph=True, async_exec=form != "bsp")
            bt.solve(b, x, stream)
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                bt.solve(b, x, stream)
            e1.record(stream)
            stream.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if bt.status() != 0:
                bt.close()
                continue
            times[f"{form}/{pc}"] = ms
            if best is None or ms < best[1]:
                if best is not None:
                    best[0].close()
                best = (bt, ms, form, pc)
            else:
                bt.close()
    if best is None:
        raise RuntimeError("no batch configuration completed without a device error")
    bt, ms, form, pc = best
    entry = {"form": form, "per_claim": pc, "ms": times}
    if path:
        table = load_table(path)
        table[key] = entry
        store_table(path, table)
    return bt, entry
