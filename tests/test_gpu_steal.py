"""The persistent solve's robbing of workgroups that have not started (lane
and wavefront cores): every 7th workgroup is made to start late (the start
delay diagnostic), the others rob it after a short wait, and the late ones
find themselves robbed and claim what is left of their first superstep, so
items are claimed by owners and thieves in racing order.  Every result is
bit-identical to the oracle, over repeated solves (each solve has its own
epoch), with other work on another stream, and when the solve is captured in
a hipGraph and replayed (the epoch comes from the per-launch start ticket,
not from the launch arguments)."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def systems():
    return [gen.erdos_renyi(120_000, 4e-5, gen.SEED_BASE + 950), gen.stencil_2d5(200, 150),
            gen.narrow_band(40_000, 0.14, 10.0, gen.SEED_BASE + 951), gen.stencil_3d7(30)]


OPTS = {"growlocal": lambda: B.gpu_opts(), "wavefront": lambda: B.default_opts(schedule_kind=B.SCHED_WAVEFRONT),
        "wave_cores": lambda: B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)}


@pytest.mark.parametrize("name", sorted(OPTS))
@pytest.mark.parametrize("steal_us,delay_us", [(0, 0), (0, 150), (20, 400)])
def test_stealing_is_exact(name, steal_us, delay_us):
    import torch
    side = torch.cuda.Stream()
    for m in systems():
        b = gen.rhs_uniform(m.n, 9)
        want = oracle.solve(m, b)
        bd = torch.from_numpy(b).cuda()
        with B.Plan(m, OPTS[name]()) as plan:
            plan.set_steal_wait(steal_us)
            plan.set_start_delay(delay_us)
            print(f"steal: {m.name} {name} steal_us={steal_us} delay_us={delay_us} "
                  f"S={plan.info()['supersteps']}", flush=True)
            for rep in range(4):
                x = torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda")
                if rep == 3:   # with other kernels queued on another stream
                    with torch.cuda.stream(side):
                        a = torch.randn(1 << 22, device="cuda")
                        for _ in range(30):
                            a = torch.sin(a) + 1.0
                plan.solve(bd, x)
                torch.cuda.synchronize()
                assert plan.device_status() == 0, (m.name, name, rep)
                assert oracle.same_bits(x.cpu().numpy(), want), (m.name, name, rep)


@pytest.mark.parametrize("name", sorted(OPTS))
def test_persistent_solve_in_a_graph(name):
    import torch
    m = gen.erdos_renyi(60_000, 1e-4, gen.SEED_BASE + 960)
    bs = [gen.rhs_uniform(m.n, 20 + r) for r in range(4)]
    with B.Plan(m, OPTS[name]()) as plan:
        plan.set_steal_wait(0)
        plan.set_start_delay(100)
        stream = torch.cuda.Stream()
        bd = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        x = torch.zeros_like(bd)
        with torch.cuda.stream(stream):
            plan.solve(bd, x, stream)          # warm-up outside the capture
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            plan.solve(bd, x, stream)
        for r, b in enumerate(bs):
            bd.copy_(torch.from_numpy(b))
            x.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert plan.device_status() == 0, (name, r)
            assert oracle.same_bits(x.cpu().numpy(), oracle.solve(m, b)), (name, r)
            # eager work between the replays
            plan.solve(bd, torch.empty_like(x))
            torch.cuda.synchronize()


@pytest.mark.parametrize("name", sorted(OPTS))
@pytest.mark.parametrize("delay_us", [0, 1500])
def test_semi_async_robbing_is_exact(name, delay_us):
    """Semi-asynchronous forms with every 7th workgroup starting late: waves
    that wait past the rob limit run the late workgroups' chunks or tasks
    (which the late ones run again on starting) -- same bits."""
    import torch
    for m in systems():
        b = gen.rhs_uniform(m.n, 19)
        want = oracle.solve(m, b)
        bd = torch.from_numpy(b).cuda()
        with B.Plan(m, OPTS[name]()) as plan:
            plan.set_start_delay(delay_us)
            print(f"semi-async robbing: {m.name} {name} delay_us={delay_us}", flush=True)
            for rep in range(2):
                x = torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda")
                plan.solve_async(bd, x)
                torch.cuda.synchronize()
                assert plan.device_status() == 0, (m.name, name, rep)
                assert oracle.same_bits(x.cpu().numpy(), want), (m.name, name, rep)
            if OPTS[name]().core_width != 64:
                cols = torch.stack([bd, -bd, 2 * bd, bd], dim=1).contiguous()
                X = plan.solve_multi(cols)
                torch.cuda.synchronize()
                assert plan.device_status() == 0
                assert oracle.same_bits(X[:, 0].cpu().numpy(), want), (m.name, name, "multi")
                assert oracle.same_bits(X[:, 3].cpu().numpy(), want), (m.name, name, "multi")
