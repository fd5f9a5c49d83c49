"""The no-allocation batched solve (gltrsv_solve_batched_noalloc): through the
C ABI, its x is bit-identical to gltrsv_solve_batched's (and to the oracle's)
on two calls in a row, the second with a smaller batch, so the state left in
the library's fixed device array by the first call is cleared before the
second uses it; a batch beyond the array's limits is refused."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _systems(count, seed):
    ms = gen.batch_mix(count, seed=seed, lo_exp=2.0, hi_exp=4.5)
    ms += [gen.narrow_band(3000, 0.03, 42.0, seed + 1), gen.edgeless(77), gen.chain(150)]
    return ms


def _plans(ms):
    return [B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT) if i % 3 == 0 else B.gpu_opts())
            for i, m in enumerate(ms)]


@pytest.mark.parametrize("in_place", [False, True])
def test_noalloc_equals_allocating_batched_solve(in_place):
    import torch
    big, small = _systems(24, gen.SEED_BASE + 700), _systems(5, gen.SEED_BASE + 710)
    for call, ms in enumerate((big, small)):
        print(f"no-alloc call {call}: {len(ms)} systems, {sum(m.n for m in ms)} rows, in_place={in_place}",
              flush=True)
        plans = _plans(ms)
        try:
            bs = [gen.rhs_uniform(m.n, 50 * call + i) for i, m in enumerate(ms)]
            ref = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
            B.solve_batched(plans, [torch.from_numpy(b).cuda() for b in bs], ref)
            if in_place:
                xs = [torch.from_numpy(b).cuda() for b in bs]
                B.solve_batched_noalloc(plans, xs, xs)
            else:
                xs = [torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda") for m in ms]
                B.solve_batched_noalloc(plans, [torch.from_numpy(b).cuda() for b in bs], xs)
            torch.cuda.synchronize()
            for i, m in enumerate(ms):
                got = xs[i].cpu().numpy()
                assert np.array_equal(got.view(np.uint64), ref[i].cpu().numpy().view(np.uint64)), (call, m.name)
                assert oracle.same_bits(got, oracle.solve(m, bs[i])), (call, m.name)
        finally:
            for p in plans:
                p.close()


def test_noalloc_refuses_batches_beyond_its_array():
    import torch
    m = gen.chain(100_000)            # wavefront schedule: one superstep per row
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)) as plan:
        assert plan.info()["supersteps"] == m.n
        b = torch.ones(m.n, dtype=torch.float64, device="cuda")
        # 11 systems of 1e5 supersteps need 4.4 MB of done counters
        xs = [torch.empty_like(b) for _ in range(11)]
        with pytest.raises(B.GltrsvError) as e:
            B.solve_batched_noalloc([plan] * 11, [b] * 11, xs)
        assert e.value.code == -5
    tiny = [B.Plan(gen.edgeless(1), B.gpu_opts()) for _ in range(1025)]
    try:
        b1 = torch.ones(1, dtype=torch.float64, device="cuda")
        x1 = [torch.empty_like(b1) for _ in tiny]
        with pytest.raises(B.GltrsvError) as e:
            B.solve_batched_noalloc(tiny, [b1] * len(tiny), x1)
        assert e.value.code == -5
    finally:
        for p in tiny:
            p.close()
    # a small batch still runs after the refusal
    small = [gen.edgeless(10), gen.fig_1_1()]
    ps = [B.Plan(q, B.gpu_opts()) for q in small]
    try:
        bs = [torch.ones(q.n, dtype=torch.float64, device="cuda") for q in small]
        xs = [torch.empty_like(v) for v in bs]
        B.solve_batched_noalloc(ps, bs, xs)
        for q, v in zip(small, xs):
            assert oracle.same_bits(v.cpu().numpy(), oracle.solve(q, np.ones(q.n)))
    finally:
        for p in ps:
            p.close()


def test_noalloc_rejects_overlapping_vectors():
    import torch
    ms = [gen.edgeless(100), gen.edgeless(100)]
    ps = [B.Plan(q, B.gpu_opts()) for q in ms]
    try:
        buf = torch.ones(150, dtype=torch.float64, device="cuda")
        b0, x1 = buf[:100], buf[50:150]
        x0 = torch.empty(100, dtype=torch.float64, device="cuda")
        b1 = torch.ones(100, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError):
            B.solve_batched_noalloc(ps, [b0, b1], [x0, x1])     # system 1's x overlaps system 0's b
    finally:
        for p in ps:
            p.close()
