"""Property tests of every device form (GPU): on random small DAGs and random
plan options (schedule kind and parameters, core width, triangle, reorder
kept or not, packing on host or device), the persistent, plain,
semi-asynchronous, several-right-hand-side and no-reorder solves all give
the oracle's bits; so do batches of random systems in every batched form
(BSP, semi-asynchronous, semi-asynchronous on wavefront cores) on grids of
one workgroup up to the default.  Hypothesis draws the cases and shrinks
any failure."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


@st.composite
def cases(draw):
    n = draw(st.integers(1, 300))
    density = draw(st.sampled_from([0.0, 0.01, 0.05, 0.2, 0.6]))
    band = draw(st.sampled_from([None, 3, 12]))
    m = gen.random_lower(n, density, draw(st.integers(0, 2 ** 31 - 1)), band=band)
    upper = draw(st.booleans())
    opts = dict(
        k=draw(st.sampled_from([1, 2, 5, 64, 1 << 16])),
        L=draw(st.sampled_from([0.0, 10.0, 50.0, 500.0])),
        alpha0=draw(st.sampled_from([1.0, 20.0])),
        schedule_kind=draw(st.sampled_from([B.SCHED_GROWLOCAL, B.SCHED_WAVEFRONT, B.SCHED_AUTO])),
        core_width=draw(st.sampled_from([1, 64])),
        reorder=draw(st.sampled_from([0, 1])),
        pack=draw(st.sampled_from([B.PACK_HOST, B.PACK_DEVICE])),
        blocks=draw(st.sampled_from([0, 0, 3])),
        triangle=B.UPPER if upper else B.LOWER,
    )
    return (gen.upper_of(m) if upper else m), opts, draw(st.integers(0, 1000))


@settings(max_examples=2000, deadline=None, suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(cases())
def test_every_form_matches_the_oracle(case):
    import torch
    m, opts, seed = case
    upper = opts["triangle"] == B.UPPER
    b = gen.rhs_uniform(m.n, seed)
    want = oracle.solve_upper(m, b) if upper else oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, B.default_opts(**opts)) as plan:
        forms = [plan.solve, plan.solve_plain, plan.solve_async]
        if opts["reorder"] == 0:
            forms.append(plan.solve_unordered)
        for solve in forms:
            x = torch.full_like(bd, float("nan"))
            solve(bd, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), (solve.__name__, opts)
        X = plan.solve_multi(torch.stack([bd, 2 * bd], dim=1).contiguous())
        torch.cuda.synchronize()
        assert oracle.same_bits(X[:, 0].cpu().numpy(), want), ("multi", opts)
        want2 = oracle.solve_upper(m, 2 * b) if upper else oracle.solve(m, 2 * b)
        assert oracle.same_bits(X[:, 1].cpu().numpy(), want2), ("multi", opts)


@st.composite
def batches(draw):
    count = draw(st.integers(1, 6))
    width = draw(st.sampled_from([1, 64]))
    systems = []
    for _ in range(count):
        n = draw(st.integers(1, 200))
        m = gen.random_lower(n, draw(st.sampled_from([0.0, 0.02, 0.1, 0.4])), draw(st.integers(0, 2 ** 31 - 1)),
                             band=draw(st.sampled_from([None, 4])))
        upper = draw(st.booleans())
        kind = draw(st.sampled_from([B.SCHED_GROWLOCAL, B.SCHED_WAVEFRONT]))
        systems.append((gen.upper_of(m) if upper else m, dict(schedule_kind=kind, k=draw(st.sampled_from([1, 3, 64])),
                                                          L=10.0, alpha0=1.0, core_width=width,
                                                          triangle=B.UPPER if upper else B.LOWER)))
    form = draw(st.sampled_from(["bsp", "async"]))
    return systems, form, draw(st.integers(1, 3)), draw(st.sampled_from([0, 1, 3]))


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(batches())
def test_every_batch_form_matches_the_oracle(case):
    import torch
    systems, form, per_claim, grid = case
    plans = [B.Plan(m, B.default_opts(**o)) for m, o in systems]
    try:
        bs = [gen.rhs_uniform(m.n, i) for i, (m, _) in enumerate(systems)]
        wants = [(oracle.solve_upper if o["triangle"] == B.UPPER else oracle.solve)(m, b)
                 for (m, o), b in zip(systems, bs)]
        bd = [torch.from_numpy(b).cuda() for b in bs]
        xd = [torch.full_like(v, float("nan")) for v in bd]
        with B.Batch(plans, per_claim=per_claim, grid_blocks=grid, use_graph=False,
                     async_exec=form == "async") as bt:
            bt.solve(bd, xd)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for (m, o), x, w in zip(systems, xd, wants):
            assert oracle.same_bits(x.cpu().numpy(), w), (m.name, o, form)
    finally:
        for p in plans:
            p.close()
