"""Batched solves (many systems, one persistent launch): every system's x is
bit-identical to the oracle's, alone or in the batch, for several claim
sizes, with and without hipGraph replay (replays interleaved with other
device work, each one checked)."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def systems():
    ms = gen.small_set(3000)
    ms += [gen.fig_1_1(), gen.edgeless(70), gen.chain(130), gen.random_lower(65, 0.1, 3)]
    kinds = [B.gpu_opts()] * len(ms)
    ms += [gen.stencil_2d5(30, 20), gen.stencil_3d7(9)]
    kinds += [B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)] * 2
    ms.append(gen.narrow_band(2000, 0.03, 42.0, 5))
    kinds.append(B.default_opts(k=8, L=20.0))
    return ms, kinds


@pytest.fixture(scope="module")
def plans():
    ms, kinds = systems()
    ps = [B.Plan(m, o) for m, o in zip(ms, kinds)]
    yield ms, ps
    for p in ps:
        p.close()


@pytest.mark.parametrize("async_exec", [False, True])
@pytest.mark.parametrize("per_claim", [1, 4])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_oracle(plans, per_claim, use_graph, async_exec):
    import torch
    ms, ps = plans
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with B.Batch(ps, per_claim=per_claim, use_graph=use_graph, async_exec=async_exec) as bt:
            assert bt.info()["systems"] == len(ps)
            for rep in range(3):
                bs = [gen.rhs_uniform(m.n, 100 * rep + i) for i, m in enumerate(ms)]
                bd = [torch.from_numpy(b).cuda() for b in bs]
                xd = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
                bt.solve(bd, xd, stream)
                stream.synchronize()
                assert bt.status() == 0
                for i, m in enumerate(ms):
                    assert oracle.same_bits(xd[i].cpu().numpy(), oracle.solve(m, bs[i])), (rep, m.name)
                # unrelated device work between replays
                junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
                (junk * 2).sum().item()


def test_one_shot_and_in_place(plans):
    import torch
    ms, ps = plans
    bs = [gen.rhs_ones(m.n) for m in ms]
    xd = [torch.from_numpy(b).cuda() for b in bs]       # b aliases x
    B.solve_batched(ps, xd, xd)
    for i, m in enumerate(ms):
        assert oracle.same_bits(xd[i].cpu().numpy(), oracle.solve(m, bs[i])), m.name


def test_batch_mix_small():
    """The batching workload generator at small sizes (n = 10^2..10^4)."""
    import torch
    ms = gen.batch_mix(12, lo_exp=2.0, hi_exp=4.0)
    ps = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT) if m.meta.get("family") == "stencil"
                 else B.gpu_opts()) for m in ms]
    bs = [gen.rhs_uniform(m.n, i) for i, m in enumerate(ms)]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    xd = [torch.empty_like(b) for b in bd]
    with B.Batch(ps, per_claim=2) as bt:
        bt.solve(bd, xd)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for i, m in enumerate(ms):
        assert oracle.same_bits(xd[i].cpu().numpy(), oracle.solve(m, bs[i])), m.name
    for p in ps:
        p.close()


def test_async_batch_rejects_in_place(plans):
    import torch
    ms, ps = plans
    xd = [torch.from_numpy(gen.rhs_ones(m.n)).cuda() for m in ms]
    with B.Batch(ps, async_exec=True) as bt:
        with pytest.raises(B.GltrsvError):
            bt.solve(xd, xd)


def test_async_batch_mix_small():
    import torch
    ms = gen.batch_mix(12, lo_exp=2.0, hi_exp=4.0)
    ps = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) for m in ms]
    bs = [gen.rhs_uniform(m.n, i) for i, m in enumerate(ms)]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    xd = [torch.empty_like(b) for b in bd]
    for per_claim in (1, 3):
        with B.Batch(ps, per_claim=per_claim, async_exec=True) as bt:
            bt.solve(bd, xd)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for i, m in enumerate(ms):
            assert oracle.same_bits(xd[i].cpu().numpy(), oracle.solve(m, bs[i])), (m.name, per_claim)
    for p in ps:
        p.close()


@pytest.mark.parametrize("async_exec", [False, True])
def test_shuffled_system_order_and_grid_sizes(plans, async_exec):
    # the systems listed in random orders (so waves start their scans at
    # different systems and claim chunks in different interleavings) on grids
    # of 1, 3 and 17 workgroups and the default: every x is the same bits
    import torch
    ms, ps = plans
    bs = [gen.rhs_uniform(m.n, 7 + i) for i, m in enumerate(ms)]
    wants = [oracle.solve(m, b) for m, b in zip(ms, bs)]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    rng = np.random.default_rng(11)
    for trial, grid in enumerate((1, 3, 17, 0)):
        order = rng.permutation(len(ms))
        xd = [torch.full((ms[i].n,), float("nan"), dtype=torch.float64, device="cuda") for i in order]
        with B.Batch([ps[i] for i in order], per_claim=1 + trial % 2, grid_blocks=grid,
                     async_exec=async_exec) as bt:
            if grid:
                assert bt.info()["grid_blocks"] <= grid
            bt.solve([bd[i] for i in order], xd)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for j, i in enumerate(order):
            assert oracle.same_bits(xd[j].cpu().numpy(), wants[i]), (grid, ms[i].name)


@pytest.mark.parametrize("per_claim", [1, 3])
@pytest.mark.parametrize("grid", [1, 5, 0])
@pytest.mark.parametrize("use_graph", [False, True])
def test_wave_core_async_batch(per_claim, grid, use_graph):
    # every plan with core width 64: the batch runs on wavefront cores (tasks
    # claimed in order per system); every x is the oracle's bits, on grids of
    # one workgroup up to the default, with and without graph replay
    import torch
    ms, _ = systems()
    ps = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT if i % 2 else B.SCHED_GROWLOCAL,
                                   core_width=64, k=256)) for i, m in enumerate(ms)]
    bs = [gen.rhs_uniform(m.n, 300 + i) for i, m in enumerate(ms)]
    wants = [oracle.solve(m, b) for m, b in zip(ms, bs)]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    with B.Batch(ps, per_claim=per_claim, use_graph=use_graph, grid_blocks=grid, async_exec=True) as bt:
        for rep in range(2):
            xd = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
            bt.solve(bd, xd)
            torch.cuda.synchronize()
            assert bt.status() == 0
            for i, m in enumerate(ms):
                assert oracle.same_bits(xd[i].cpu().numpy(), wants[i]), (rep, m.name)
    # a mix of core widths falls back to lane cores (the stream every plan keeps)
    mixed = ps[:3] + [B.Plan(ms[3], B.gpu_opts())]
    xd = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms[:4]]
    with B.Batch(mixed, async_exec=True) as bt:
        bt.solve(bd[:4], xd)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for i in range(4):
        assert oracle.same_bits(xd[i].cpu().numpy(), wants[i])
    for p in ps + mixed[3:]:
        p.close()


def test_wave_core_batch_mixes_forward_and_backward_systems():
    import torch
    lows = [gen.erdos_renyi(2500, 0.004, gen.SEED_BASE + 70), gen.narrow_band(2000, 0.1, 12, gen.SEED_BASE + 71)]
    ups = [gen.upper_of(m) for m in lows]
    ms = lows + ups
    ps = [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT, core_width=64,
                                   triangle=B.UPPER if m.meta.get("upper") else B.LOWER)) for m in ms]
    bs = [gen.rhs_uniform(m.n, 40 + i) for i, m in enumerate(ms)]
    wants = [(oracle.solve_upper if m.meta.get("upper") else oracle.solve)(m, b) for m, b in zip(ms, bs)]
    bd = [torch.from_numpy(b).cuda() for b in bs]
    xd = [torch.full_like(v, float("nan")) for v in bd]
    with B.Batch(ps, async_exec=True) as bt:
        bt.solve(bd, xd)
        torch.cuda.synchronize()
        assert bt.status() == 0
    for m, x, w in zip(ms, xd, wants):
        assert oracle.same_bits(x.cpu().numpy(), w), m.name
    for p in ps:
        p.close()
