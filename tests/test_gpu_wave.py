"""Wavefront cores (GPU): with opts.core_width = 64 a BSP core is a whole
wavefront that forms 64 products of a row at once and subtracts them in
stored order.  gltrsv_solve, gltrsv_solve_plain and gltrsv_solve_async
(semi-asynchronous wave cores) must give the oracle's
bits for lower and upper systems, rows shorter and longer than 64 entries,
same-task dependencies near (LDS ring) and far (memory) and every schedule
kind, in place or not; several right-hand sides keep lane cores."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

CASES = [
    ("dense_rows", lambda: gen.erdos_renyi(3000, 0.05, gen.SEED_BASE + 61)),      # ~75 entries a row
    ("er", lambda: gen.erdos_renyi(6000, 0.002, gen.SEED_BASE + 62)),
    ("one_task", lambda: gen.random_lower(700, 0.08, 63)),                        # k = 1: dependencies at every distance
    ("chain", lambda: gen.chain(300)),
    ("grid", lambda: gen.stencil_3d7(12)),
    ("fig1_1", gen.fig_1_1),
    ("edgeless", lambda: gen.edgeless(500)),
    ("very_long_rows", lambda: gen.random_lower(400, 0.9, 64)),                  # up to ~360 entries a row
]
OPTS = [
    ("k1024", dict(k=1024, L=50.0, alpha0=1.0)),
    ("k1", dict(k=1)),
    ("wavefront", dict(schedule_kind=B.SCHED_WAVEFRONT)),
    ("auto", dict(schedule_kind=B.SCHED_AUTO, k=1024, L=50.0, alpha0=1.0)),
]


@pytest.mark.parametrize("oname", [o[0] for o in OPTS])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
@pytest.mark.parametrize("upper", [False, True])
def test_wave_cores_match_the_oracle(case, oname, upper):
    import torch
    m = dict(CASES)[case]()
    over = dict(dict(OPTS)[oname])
    if upper:
        m = gen.upper_of(m)
        over["triangle"] = B.UPPER
    b = gen.rhs_uniform(m.n, 4)
    want = oracle.solve_upper(m, b) if upper else oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, B.default_opts(core_width=64, **over)) as plan:
        assert plan.info()["core_width"] == 64
        for solve in (plan.solve, plan.solve_plain, plan.solve_async):
            x = torch.full_like(bd, float("nan"))
            solve(bd, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), solve.__name__
            y = bd.clone()
            solve(y, y)
            torch.cuda.synchronize()
            assert oracle.same_bits(y.cpu().numpy(), want), ("in place", solve.__name__)
        X = plan.solve_multi(torch.stack([bd, -bd], dim=1).contiguous())   # lane cores, same schedule
        torch.cuda.synchronize()
        assert oracle.same_bits(X[:, 0].cpu().numpy(), want)


def test_wave_cores_repeat_and_reject_bad_width():
    import torch
    m = gen.erdos_renyi(5000, 0.02, gen.SEED_BASE + 65)
    want = oracle.solve(m, np.ones(m.n))
    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    with B.Plan(m, B.default_opts(core_width=64, k=1024, L=50.0, alpha0=1.0)) as plan:
        x = torch.empty_like(b)
        for solve in (plan.solve, plan.solve_async):
            for _ in range(30):
                x.fill_(float("nan"))
                solve(b, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want)
    with pytest.raises(B.GltrsvError):
        B.Plan(m, B.default_opts(core_width=32))
