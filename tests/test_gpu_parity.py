"""GPU parity: every solve path of the HIP library against the CPU oracle,
bit for bit (binary64, sign of zero included; NaNs equal by class).

Each x_i has exactly one correct value under the fixed per-row operation
order (running subtraction in stored order, no fused multiply-add, one
correctly rounded division), whatever the schedule, so the tolerance is 0 ULP.
"""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _solve_both(m, opts, b=None, seed=0):
    torch = _torch()
    b = gen.rhs_uniform(m.n, seed) if b is None else b
    want = oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, opts) as plan:
        x1 = plan.solve(bd)
        x2 = plan.solve_plain(bd)
        x3 = plan.solve_async(bd)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        info = plan.info()
    # the semi-asynchronous form (no barriers) computes the same bits
    assert oracle.same_bits(x3.cpu().numpy(), want), (m.name, "async")
    return want, x1.cpu().numpy(), x2.cpu().numpy(), info


OPTS = {
    "paper": dict(),
    "gpu": dict(k=1 << 16, L=50.0, alpha0=1.0),
    "k3": dict(k=3, L=0.0),
    "wavefront": dict(schedule_kind=B.SCHED_WAVEFRONT),
    "auto": dict(k=1 << 16, L=50.0, alpha0=1.0, schedule_kind=B.SCHED_AUTO),
}


@pytest.mark.parametrize("optname", list(OPTS))
@pytest.mark.parametrize("idx", range(6))
def test_small_set(idx, optname):
    m = gen.small_set()[idx]
    # (with the paper's parameters ER n = 1e4, p = 0.02 gets a serial schedule, S = 1: one lane walks
    # all 2e6 entries, a fraction of a second per solve)
    want, x1, x2, info = _solve_both(m, B.default_opts(**OPTS[optname]), seed=idx)
    print(m.name, optname, info["supersteps"], info["chunks"], flush=True)
    assert oracle.same_bits(x1, want)
    assert oracle.same_bits(x2, want)


@pytest.mark.parametrize("maker", [
    lambda: gen.fig_1_1(), lambda: gen.fig_3_1(), lambda: gen.edgeless(1), lambda: gen.edgeless(65),
    lambda: gen.edgeless(1000), lambda: gen.chain(2), lambda: gen.chain(257), lambda: gen.stencil_2d5(17, 5),
    lambda: gen.random_lower(63, 0.2, 7), lambda: gen.random_lower(64, 0.05, 8), lambda: gen.random_lower(200, 0.3, 9),
    lambda: gen.random_lower(300, 0.02, 10, band=4),
], ids=["fig1_1", "fig3_1", "n1", "edgeless65", "edgeless1000", "chain2", "chain257", "grid17x5", "r63", "r64",
        "r200", "band300"])
@pytest.mark.parametrize("optname", list(OPTS))
def test_edge_shapes(maker, optname):
    m = maker()
    want, x1, x2, _ = _solve_both(m, B.default_opts(**OPTS[optname]))
    assert oracle.same_bits(x1, want)
    assert oracle.same_bits(x2, want)


def test_in_place_and_repeat():
    torch = _torch()
    m = gen.small_set()[3]
    b = gen.rhs_uniform(m.n, 3)
    want = oracle.solve(m, b)
    with B.Plan(m, B.gpu_opts()) as plan:
        for rep in range(5):
            xb = torch.from_numpy(b).cuda()
            plan.solve(xb, xb)          # b aliases x
            torch.cuda.synchronize()
            assert oracle.same_bits(xb.cpu().numpy(), want), rep
        assert plan.device_status() == 0


def test_poisoned_output():
    """x pre-filled with NaN: any read of a not-yet-computed value would
    propagate a NaN into the result."""
    torch = _torch()
    m = gen.small_set()[0]
    b = gen.rhs_ones(m.n)
    want = oracle.solve(m, b)
    with B.Plan(m, B.gpu_opts()) as plan:
        x = torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda")
        plan.solve(torch.from_numpy(b).cuda(), x)
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
        x.fill_(float("nan"))
        plan.solve_plain(torch.from_numpy(b).cuda(), x)
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)


@pytest.mark.parametrize("nblocks", [2, 7])
def test_block_parallel_schedule_solves_exactly(nblocks):
    for m in (gen.random_lower(6000, 0.003, 41), gen.narrow_band(20000, 0.05, 20, 6)):
        want, x1, x2, info = _solve_both(m, B.gpu_opts(blocks=nblocks), seed=nblocks)
        pi, sg, S = oracle.growlocal_blocks(m, 1 << 16, nblocks, L=50.0, alpha0=1.0)
        assert info["supersteps"] == S
        assert oracle.same_bits(x1, want) and oracle.same_bits(x2, want), m.name


def test_async_in_place_and_repeated():
    import torch
    m = gen.narrow_band(30000, 0.05, 20, 8)
    b = gen.rhs_uniform(m.n, 4)
    want = oracle.solve(m, b)
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_WAVEFRONT)) as plan:
        for rep in range(3):
            x = torch.from_numpy(b).cuda()
            plan.solve_async(x, x)          # in place: b == x
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), rep
        bd = torch.from_numpy(b).cuda()
        x = torch.empty_like(bd)
        for rep in range(3):
            plan.solve_async(bd, x)
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)


@pytest.mark.parametrize("cap", [8, 64])
def test_funnel_schedule_solves_exactly(cap):
    for m in (gen.random_lower(6000, 0.003, 43), gen.narrow_band(20000, 0.05, 20, 7), gen.stencil_2d5(80, 50)):
        want, x1, x2, info = _solve_both(m, B.gpu_opts(funnel_max_weight=cap), seed=cap)
        pi, sg, S, _ = oracle.funnel_growlocal(m, 1 << 16, cap, L=50.0, alpha0=1.0)
        assert info["supersteps"] == S
        assert oracle.same_bits(x1, want) and oracle.same_bits(x2, want), m.name


def test_auto_for_async_execution_picks_the_lower_prediction():
    import torch
    for m in (gen.narrow_band(20000, 0.03, 42, 11), gen.erdos_renyi_paper(20000, 1e-4, gen.SEED_BASE + 5),
              gen.stencil_2d5(90, 60)):
        pred = {}
        for kind in (B.SCHED_GROWLOCAL, B.SCHED_WAVEFRONT, B.SCHED_AUTO):
            with B.Plan(m, B.gpu_opts(schedule_kind=kind, exec_hint=1)) as plan:
                inf = plan.info()
                pred[kind] = (inf["predicted_us"], inf["schedule_kind"])
                if kind == B.SCHED_AUTO:
                    b = torch.from_numpy(gen.rhs_uniform(m.n, 2)).cuda()
                    x = plan.solve_async(b)
                    torch.cuda.synchronize()
                    assert oracle.same_bits(x.cpu().numpy(), oracle.solve(m, b.cpu().numpy()))
        best = min(pred[B.SCHED_GROWLOCAL][0], pred[B.SCHED_WAVEFRONT][0])
        assert pred[B.SCHED_AUTO][0] == best, (m.name, pred)


def test_watchdog_reports_a_forced_timeout_and_the_plan_recovers():
    # a spin limit of one poll, forced from the host: some barrier / readiness
    # wait of this 118-level grid takes longer, the solve sets the error word,
    # every wave leaves normally, the status reports it once, and the plan
    # solves exactly again with the default limit
    import torch
    m = gen.stencil_3d7(40)
    b = gen.rhs_uniform(m.n, 9)
    want = oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)) as plan:
        assert plan.info()["grid_blocks"] > 1
        plan.set_spin_limit(1)
        x = plan.solve(bd)
        torch.cuda.synchronize()
        assert plan.device_status() == 1
        assert plan.device_status() == 0            # reported once, then cleared
        plan.solve_async(bd, x)
        torch.cuda.synchronize()
        assert plan.device_status() == 1
        plan.set_spin_limit(5_000_000)
        for solve in (plan.solve, plan.solve_async, plan.solve_plain):
            x.fill_(float("nan"))
            solve(bd, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want)
        with pytest.raises(B.GltrsvError):
            plan.set_spin_limit(0)


def test_plan_from_a_stored_schedule(tmp_path):
    # the analysis of one process reused by another: same schedule, same
    # stream, same bits, without rescheduling; invalid schedules and other
    # patterns are refused
    import torch
    for m, opts in ((gen.random_lower(7000, 0.002, 95), B.gpu_opts()),
                    (gen.upper_of(gen.narrow_band(9000, 0.05, 20, 14)), B.gpu_opts(triangle=B.UPPER))):
        path = str(tmp_path / "sched.npz")
        b = torch.from_numpy(gen.rhs_uniform(m.n, 1)).cuda()
        with B.Plan(m, opts) as p1:
            p1.save_schedule(path)
            w1, v1 = p1.stream()
            x1 = p1.solve(b)
            core, sup, _ = p1.schedule()
        with B.Plan.load_schedule(m, path, opts) as p2:
            assert p2.info()["schedule_kind"] == B.SCHED_GIVEN
            w2, v2 = p2.stream()
            x2 = p2.solve(b)
            torch.cuda.synchronize()
            assert np.array_equal(w1, w2) and np.array_equal(v1.view(np.uint64), v2.view(np.uint64))
            assert oracle.same_bits(x1.cpu().numpy(), x2.cpu().numpy())
        bad = sup.copy()
        bad[:] = 0
        core_bad = np.arange(m.n, dtype=np.int32)        # everything in one superstep on different cores
        if m.row_ptr[-1] > m.n:
            with pytest.raises(B.GltrsvError):
                B.Plan(m, opts, schedule=(core_bad, bad))
    other = gen.random_lower(7000, 0.002, 96)
    with B.Plan(gen.random_lower(7000, 0.002, 95), B.gpu_opts()) as p1:
        p1.save_schedule(str(tmp_path / "s2.npz"))
    with pytest.raises((ValueError, B.GltrsvError)):
        B.Plan.load_schedule(other, str(tmp_path / "s2.npz"), B.gpu_opts())
