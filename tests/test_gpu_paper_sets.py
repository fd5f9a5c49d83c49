"""Parity at the paper's sizes: the Erdos-Renyi and narrow-band sets of
Sec. 6.2 (Tables A.4, A.5; n = 1e5, ten seeds each) solved singly and as one
batch (lane and wavefront cores), and the n = 1e7 workloads, every x
bit-identical to the oracle's.  Also records supersteps against wavefronts (the quantity of
Table 7.2) for the GPU schedules."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

FAMILIES = [("ER", p) for p in gen.ER_PROBS] + [("NB", pb) for pb in gen.NB_PAIRS]


def make(family, param, i):
    if family == "ER":
        return gen.erdos_renyi_paper(100_000, param, gen.SEED_BASE + i)
    return gen.narrow_band(100_000, param[0], param[1], gen.SEED_BASE + 10 + i)


@pytest.mark.parametrize("fam", range(len(FAMILIES)), ids=[f"{f}{p}" for f, p in FAMILIES])
def test_paper_set_single_and_batched(fam):
    import torch
    family, param = FAMILIES[fam]
    seeds = range(10) if not (family == "ER" and param == 2e-3) else range(3)   # 2e7 entries each
    ms = [make(family, param, i) for i in seeds]
    plans = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) for m in ms]
    wants = [oracle.solve(m, np.ones(m.n)) for m in ms]
    bd = [torch.ones(m.n, dtype=torch.float64, device="cuda") for m in ms]
    for m, p, want, b in zip(ms, plans, wants, bd):
        x = p.solve(b)
        torch.cuda.synchronize()
        assert p.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want), m.name
        inf = p.info()
        print(f"{m.name} S={inf['supersteps']} wavefronts={inf['wavefronts']} "
              f"ratio={inf['wavefronts'] / inf['supersteps']:.2f} kind={inf['schedule_kind']}", flush=True)
    xd = [torch.full_like(b, float("nan")) for b in bd]
    with B.Batch(plans, per_claim=2) as bt:
        bt.solve(bd, xd)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for m, x, want in zip(ms, xd, wants):
        assert oracle.same_bits(x.cpu().numpy(), want), m.name
    for p in plans:
        p.close()
    # wavefront cores on the wavefront schedule: each system alone (semi-async) and all in one batch
    wplans = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) for m in ms]
    for m, p, want, b in zip(ms, wplans, wants, bd):
        x = p.solve_async(b)
        torch.cuda.synchronize()
        assert p.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want), ("wave", m.name)
    xd = [torch.full_like(b, float("nan")) for b in bd]
    with B.Batch(wplans, async_exec=True) as bt:
        bt.solve(bd, xd)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for m, x, want in zip(ms, xd, wants):
        assert oracle.same_bits(x.cpu().numpy(), want), ("wave batch", m.name)
    for p in wplans:
        p.close()


def _schedule_key(plan):
    import hashlib
    h = hashlib.sha256()
    for a in plan.schedule():          # core, superstep, perm per row
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def test_full_size_single_system():
    """The n = 1e7 workload of the benchmark: the plan's GrowLocal schedule
    and Sec. 5 order equal the oracle's (the stored key of
    tests/golden/schedule_keys.json), and the persistent, plain,
    semi-asynchronous and several-column solves, and the semi-asynchronous
    solve on wavefront cores, equal the full oracle solve."""
    import json
    import os
    import torch
    n = 10_000_000
    m = gen.erdos_renyi(n, 20.0 / (n - 1), gen.SEED_BASE + 200)
    want = oracle.solve(m, np.ones(n))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "schedule_keys.json")) as f:
        golden = json.load(f)["bench_er_n1e7"]
    assert (golden["n"], golden["nnz"]) == (m.n, m.nnz)
    with B.Plan(m, B.gpu_opts()) as p:
        assert p.info()["supersteps"] == golden["S"]
        assert _schedule_key(p) == golden["key"]
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        x = torch.full_like(b, float("nan"))
        p.solve(b, x)
        torch.cuda.synchronize()
        assert p.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)
        x.fill_(float("nan"))
        p.solve_plain(b, x)
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
        p.solve_async(b, x)
        torch.cuda.synchronize()
        assert p.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)
        X = p.solve_multi(torch.ones(n, 4, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        for r in (0, 3):
            assert oracle.same_bits(X[:, r].cpu().numpy(), want)
    # wavefront cores over per-wave record streams, at the benchmark's size
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) as p:
        x.fill_(float("nan"))
        p.solve_async(b, x)
        torch.cuda.synchronize()
        assert p.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)


@pytest.mark.parametrize("maker", [lambda: gen.stencil_3d7(216), lambda: gen.stencil_3d27(216)])
def test_full_size_grids(maker):
    """The 216^3 grids of the benchmark (AUTO schedule), persistent, plain
    and semi-asynchronous, against the full oracle solve."""
    import torch
    m = maker()
    want = oracle.solve(m, np.ones(m.n))
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) as p:
        b = torch.ones(m.n, dtype=torch.float64, device="cuda")
        x = torch.full_like(b, float("nan"))
        for solve in (p.solve, p.solve_plain, p.solve_async):
            x.fill_(float("nan"))
            solve(b, x)
            torch.cuda.synchronize()
            assert p.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), (m.name, solve.__name__)
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) as p:
        for solve in (p.solve, p.solve_async):   # wavefront cores at full size
            x.fill_(float("nan"))
            solve(b, x)
            torch.cuda.synchronize()
            assert p.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), (m.name, "wave", solve.__name__)


def test_full_size_batch_mix():
    """The 64-system batching workload (9.5e6 rows) in one launch, BSP,
    semi-asynchronous and semi-asynchronous on wavefront cores, every system
    against the oracle."""
    import torch
    ms = gen.batch_mix()
    plans = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) for m in ms]
    bs = [torch.from_numpy(gen.rhs_uniform(m.n, i)).cuda() for i, m in enumerate(ms)]
    wants = [oracle.solve(m, b.cpu().numpy()) for m, b in zip(ms, bs)]
    for async_exec in (False, True):
        xs = [torch.full_like(b, float("nan")) for b in bs]
        with B.Batch(plans, per_claim=2, async_exec=async_exec) as bt:
            bt.solve(bs, xs)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for m, x, w in zip(ms, xs, wants):
            assert oracle.same_bits(x.cpu().numpy(), w), (m.name, async_exec)
    for p in plans:
        p.close()
    wplans = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) for m in ms]
    xs = [torch.full_like(b, float("nan")) for b in bs]
    with B.Batch(wplans, async_exec=True) as bt:
        bt.solve(bs, xs)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for m, x, w in zip(ms, xs, wants):
        assert oracle.same_bits(x.cpu().numpy(), w), (m.name, "wave")
    for p in wplans:
        p.close()
