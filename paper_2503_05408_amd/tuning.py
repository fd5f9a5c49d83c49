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
