"""The schedule without the reorder of Sec. 5 (GPU): a plan created with
reorder = 0 keeps A in the caller's CSR order as well, and
gltrsv_solve_unordered walks each task's rows through the row pointers.
Results are bit-identical to the oracle and to the reordered forms for
lower and upper systems under every schedule kind; plans built with the
reorder refuse the call."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

CASES = [
    ("er", lambda: gen.erdos_renyi(5000, 0.003, gen.SEED_BASE + 51)),
    ("nb", lambda: gen.narrow_band(4000, 0.1, 12, gen.SEED_BASE + 52)),
    ("grid", lambda: gen.stencil_3d7(14)),
    ("chain", lambda: gen.chain(700)),          # one task of 700 rows: same-task reads from memory
    ("fig1_1", gen.fig_1_1),
    ("wide_rows", lambda: gen.random_lower(300, 0.6, 53)),   # rows of ~90 entries: the 4-entry loop and its tail
]
OPTS = [
    ("gpu", dict()),
    ("k3", dict(k=3, L=10.0)),
    ("wavefront", dict(schedule_kind=B.SCHED_WAVEFRONT)),
    ("auto", dict(schedule_kind=B.SCHED_AUTO)),
]


@pytest.mark.parametrize("oname", [o[0] for o in OPTS])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
@pytest.mark.parametrize("upper", [False, True])
def test_unordered_solve_matches_the_oracle(case, oname, upper):
    import torch
    m = dict(CASES)[case]()
    over = dict(dict(OPTS)[oname])
    if upper:
        m = gen.upper_of(m)
        over["triangle"] = B.UPPER
    b = gen.rhs_uniform(m.n, 3)
    want = oracle.solve_upper(m, b) if upper else oracle.solve(m, b)
    bd = torch.from_numpy(b).cuda()
    opts = B.gpu_opts(reorder=0, **over) if oname != "k3" else B.default_opts(reorder=0, **over)
    with B.Plan(m, opts) as plan:
        x = torch.full_like(bd, float("nan"))
        plan.solve_unordered(bd, x)
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
        y = bd.clone()
        plan.solve_unordered(y, y)                 # in place
        torch.cuda.synchronize()
        assert oracle.same_bits(y.cpu().numpy(), want)
        x.fill_(float("nan"))
        plan.solve(bd, x)                          # the reordered stream is still there
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)


def test_reordered_plans_refuse_and_memory_is_accounted():
    import torch
    m = gen.erdos_renyi(3000, 0.004, gen.SEED_BASE + 54)
    b = torch.ones(m.n, dtype=torch.float64, device="cuda")
    with B.Plan(m, B.gpu_opts()) as p1, B.Plan(m, B.gpu_opts(reorder=0)) as p0:
        with pytest.raises(B.GltrsvError) as ei:
            p1.solve_unordered(b)
        assert ei.value.code == -10
        extra = p0.info()["device_bytes"] - p1.info()["device_bytes"]
        assert extra >= 12 * m.nnz + 12 * m.n
