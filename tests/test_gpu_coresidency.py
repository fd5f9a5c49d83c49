"""Solves whose waves wait for each other (superstep completion, per-row
readiness across workgroups) while another stream keeps the device busy with
ordinary torch kernels, so that some workgroups of a solve start late: every
result is bit-identical to the oracle and no device-side wait runs out.

No kernel needs all of its workgroups resident (a cooperative launch does not
give that either: measured on MI355X, a cooperative grid is starved the same
way): the persistent kernels (lane and wavefront cores) rob the items of
workgroups that have not started once a superstep wait grows long, and the
semi-asynchronous kernels (lane and wavefront cores, single systems and
batches) run a chunk or task of such a workgroup in place of a long wait."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _busy(side, reps=60):
    """Queues ordinary element-wise and reduction kernels on `side`."""
    import torch
    with torch.cuda.stream(side):
        a = torch.randn(1 << 22, device="cuda", dtype=torch.float32)
        for _ in range(reps):
            a = torch.sin(a) * 1.0001 + 0.5
            a.sum()
    return a


def test_single_system_forms_with_concurrent_work():
    import torch
    ms = [gen.erdos_renyi(200_000, 2e-5, gen.SEED_BASE + 900), gen.stencil_2d5(300, 300),
          gen.narrow_band(50_000, 0.05, 20.0, gen.SEED_BASE + 901)]
    cases = [(B.gpu_opts(), ("solve", "solve_async")),
             (B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64), ("solve", "solve_async")),
             (B.gpu_opts(schedule_kind=B.SCHED_AUTO), ("solve", "solve_async", "solve_plain"))]
    side = torch.cuda.Stream()
    main = torch.cuda.Stream()
    for m in ms:
        b = gen.rhs_uniform(m.n, 5)
        want = oracle.solve(m, b)
        bd = torch.from_numpy(b).cuda()
        for opts, forms in cases:
            with B.Plan(m, opts) as plan:
                for form in forms:
                    print(f"co-residency: {m.name} core_width={opts.core_width} {form}", flush=True)
                    xs = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
                    torch.cuda.synchronize()
                    keep = _busy(side)
                    with torch.cuda.stream(main):
                        for x in xs:
                            getattr(plan, form)(bd, x, main)
                    main.synchronize()
                    side.synchronize()
                    del keep
                    assert plan.device_status() == 0, (m.name, form)
                    for x in xs:
                        assert oracle.same_bits(x.cpu().numpy(), want), (m.name, opts.core_width, form)
                if opts.core_width != 64:
                    cols = torch.stack([bd, -bd, 2 * bd], dim=1).contiguous()
                    torch.cuda.synchronize()
                    keep = _busy(side)
                    with torch.cuda.stream(main):
                        X = plan.solve_multi(cols, None, main)
                    main.synchronize()
                    side.synchronize()
                    del keep
                    assert plan.device_status() == 0, (m.name, "multi")
                    assert oracle.same_bits(X[:, 0].cpu().numpy(), want), (m.name, "multi")


@pytest.mark.parametrize("use_graph", [False, True])
def test_wave_core_batch_with_concurrent_work(use_graph):
    import torch
    ms = gen.batch_mix(10, seed=gen.SEED_BASE + 920, lo_exp=2.0, hi_exp=4.5)
    plans = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64)) for m in ms]
    side = torch.cuda.Stream()
    main = torch.cuda.Stream()
    try:
        bs = [gen.rhs_uniform(m.n, i) for i, m in enumerate(ms)]
        want = [oracle.solve(m, b) for m, b in zip(ms, bs)]
        bd = [torch.from_numpy(b).cuda() for b in bs]
        with B.Batch(plans, use_graph=use_graph, async_exec=True) as bt:
            for rep in range(3):
                xs = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
                torch.cuda.synchronize()
                keep = _busy(side)
                with torch.cuda.stream(main):
                    bt.solve(bd, xs, main)
                main.synchronize()
                side.synchronize()
                del keep
                assert bt.status() == 0, rep
                for m, x, w in zip(ms, xs, want):
                    assert oracle.same_bits(x.cpu().numpy(), w), (rep, m.name)
    finally:
        for p in plans:
            p.close()
