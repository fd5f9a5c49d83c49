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


def _every_row_length(reps, seed, longest=140):
    """160 rows without off-diagonals, then rows with every count of stored
    off-diagonals from 0 to `longest`, `reps` times over (so rows start at
    every lane of a 64-slot window and end across 16-lane rows and windows),
    columns drawn at random below the row, the paper's values."""
    rng = np.random.default_rng(seed)
    base = 160
    counts = np.tile(np.arange(longest + 1), reps)
    n = base + counts.size
    rows, cols = [], []
    for i, c in enumerate(counts):
        r = base + i
        rows.append(np.full(c, r, dtype=np.int64))
        cols.append(np.sort(rng.choice(r, size=c, replace=False)).astype(np.int64))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    off, diag = gen.paper_values(rng, rows.size, n)
    return gen._assemble(n, rows, cols, off, diag, f"every_row_length_{reps}_{seed}", presorted=True)


@pytest.mark.parametrize("upper", [False, True])
def test_both_row_subtraction_forms(upper):
    """The wave-core solves subtract a row's products through DPP lane
    broadcasts on systems of long rows and through readlane on the others;
    both give the oracle's bits on rows of every length, in every solve form
    and for a batch of each kind."""
    import torch
    long_rows = [_every_row_length(4, 81), _every_row_length(2, 82, longest=70)]
    short_rows = [gen.narrow_band(3000, 0.05, 20.0, gen.SEED_BASE + 83), gen.chain(200)]
    for group, dpp in ((long_rows, 1), (short_rows, 0)):
        ms = [gen.upper_of(m) for m in group] if upper else group
        bs = [gen.rhs_uniform(m.n, 90 + i) for i, m in enumerate(ms)]
        wants = [oracle.solve_upper(m, b) if upper else oracle.solve(m, b) for m, b in zip(ms, bs)]
        bd = [torch.from_numpy(b).cuda() for b in bs]
        tri = B.UPPER if upper else B.LOWER
        for over in (dict(schedule_kind=B.SCHED_WAVEFRONT), dict(k=4)):
            ps = [B.Plan(m, B.default_opts(core_width=64, triangle=tri, **over)) for m in ms]
            try:
                for p, b, want in zip(ps, bd, wants):
                    assert p.info()["row_dpp"] == dpp
                    for solve in (p.solve, p.solve_plain, p.solve_async):
                        x = torch.full_like(b, float("nan"))
                        solve(b, x)
                        torch.cuda.synchronize()
                        assert p.device_status() == 0
                        assert oracle.same_bits(x.cpu().numpy(), want), (p.info()["n"], over, solve.__name__)
                with B.Batch(ps, async_exec=True) as bt:
                    xd = [torch.full_like(b, float("nan")) for b in bd]
                    bt.solve(bd, xd)
                    torch.cuda.synchronize()
                    assert bt.status() == 0
                    for x, want in zip(xd, wants):
                        assert oracle.same_bits(x.cpu().numpy(), want), ("batch", over)
            finally:
                for p in ps:
                    p.close()


@pytest.mark.parametrize("width", [64, 1])
@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 129])
def test_wave_cores_at_degenerate_sizes(n, width):
    """Plans of 0, 1, 2 rows and around a window's 64 slots (wave cores, and
    lane cores for comparison), as a chain (every row waits for the one
    before) and without edges, in every solve form, and all of them in one
    semi-asynchronous batch."""
    import torch
    ms = [gen.chain(n) if n else gen.edgeless(0), gen.edgeless(n)]
    plans = [B.Plan(m, B.default_opts(core_width=width, schedule_kind=B.SCHED_WAVEFRONT)) for m in ms]
    try:
        bs = [gen.rhs_uniform(m.n, 7 + n) for m in ms]
        wants = [oracle.solve(m, b) for m, b in zip(ms, bs)]
        bd = [torch.from_numpy(b).cuda() for b in bs]
        for p, b, want in zip(plans, bd, wants):
            for solve in (p.solve, p.solve_plain, p.solve_async):
                x = torch.full_like(b, float("nan"))
                solve(b, x)
                torch.cuda.synchronize()
                assert p.device_status() == 0
                assert oracle.same_bits(x.cpu().numpy(), want), (n, solve.__name__)
        more = [B.Plan(gen.chain(70), B.default_opts(core_width=width, schedule_kind=B.SCHED_WAVEFRONT))]
        try:
            bm = [torch.from_numpy(gen.rhs_uniform(70, 3)).cuda()]
            allp, allb = plans + more, bd + bm
            allw = wants + [oracle.solve(gen.chain(70), bm[0].cpu().numpy())]
            with B.Batch(allp, async_exec=True) as bt:
                xd = [torch.full_like(b, float("nan")) for b in allb]
                bt.solve(allb, xd)
                torch.cuda.synchronize()
                assert bt.status() == 0
                for x, want in zip(xd, allw):
                    assert oracle.same_bits(x.cpu().numpy(), want), ("batch", n)
        finally:
            for p in more:
                p.close()
    finally:
        for p in plans:
            p.close()
