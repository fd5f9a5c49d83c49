"""Parity at the paper's sizes: the Erdos-Renyi and narrow-band sets of
Sec. 6.2 (Tables A.4, A.5; n = 1e5, ten seeds each) solved singly and as one
batch, and the n = 1e7 single-system workload, every x bit-identical to the
oracle's.  Also records supersteps against wavefronts (the quantity of
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


def test_full_size_single_system():
    """The n = 1e7 workload of the benchmark, persistent and plain, against
    the full oracle solve."""
    import torch
    n = 10_000_000
    m = gen.erdos_renyi(n, 20.0 / (n - 1), gen.SEED_BASE + 200)
    want = oracle.solve(m, np.ones(n))
    with B.Plan(m, B.gpu_opts()) as p:
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
