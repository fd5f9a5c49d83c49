"""Race and synchronisation checks on the GPU: every solve form gives the
same bits for any grid size (including grids far smaller than a superstep's
width and single-workgroup grids) and over many repetitions with x poisoned
(NaN) before each solve."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("grid", [1, 2, 3, 7, 64, 1000])
def test_any_grid_size_gives_the_same_bits(grid):
    import torch
    for m, o in ((gen.random_lower(9000, 0.002, 91), B.gpu_opts(grid_blocks=grid)),
                 (gen.stencil_3d7(18), B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, grid_blocks=grid))):
        b = gen.rhs_uniform(m.n, grid)
        want = oracle.solve(m, b)
        bd = torch.from_numpy(b).cuda()
        with B.Plan(m, o) as plan:
            assert plan.info()["grid_blocks"] <= grid
            for solve in (plan.solve, plan.solve_async):
                x = torch.full_like(bd, float("nan"))
                solve(bd, x)
                torch.cuda.synchronize()
                assert plan.device_status() == 0
                assert oracle.same_bits(x.cpu().numpy(), want), (m.name, grid, solve.__name__)


def test_bitwise_repeatability_with_poisoned_x():
    import torch
    m = gen.narrow_band(30000, 0.05, 20, 13)
    b = gen.rhs_uniform(m.n, 5)
    want = oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, B.gpu_opts()) as plan:
        x = torch.empty_like(bd)
        for rep in range(60):
            x.fill_(float("nan"))
            (plan.solve, plan.solve_async, plan.solve_plain)[rep % 3](bd, x)
            torch.cuda.synchronize()
            assert oracle.same_bits(x.cpu().numpy(), want), rep
        assert plan.device_status() == 0


@pytest.mark.parametrize("grid", [1, 5, 40])
def test_batch_any_grid_size(grid):
    import torch
    ms = gen.batch_mix(10, lo_exp=2.0, hi_exp=3.5, seed=gen.SEED_BASE + 300)
    plans = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) for m in ms]
    bs = [torch.from_numpy(gen.rhs_uniform(m.n, i)).cuda() for i, m in enumerate(ms)]
    for async_exec in (False, True):
        xs = [torch.full_like(b, float("nan")) for b in bs]
        with B.Batch(plans, per_claim=1, grid_blocks=grid, async_exec=async_exec) as bt:
            assert bt.info()["grid_blocks"] <= grid
            bt.solve(bs, xs)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for m, x, b in zip(ms, xs, bs):
            assert oracle.same_bits(x.cpu().numpy(), oracle.solve(m, b.cpu().numpy())), (m.name, grid, async_exec)
    for p in plans:
        p.close()
