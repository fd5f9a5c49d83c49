"""Several right-hand sides (SpTRSM): every column of X is bit-identical to
the oracle's solve of that column of B, for column counts that exercise the
4-, 2- and 1-column passes, lower and upper triangles, and several
schedules."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

GPU = dict(k=1 << 16, L=50.0, alpha0=1.0)


def _cases():
    return [
        (gen.random_lower(7000, 0.002, 61), B.default_opts(**GPU)),
        (gen.narrow_band(15000, 0.05, 20, 7), B.default_opts(**GPU)),
        (gen.stencil_2d5(70, 40), B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)),
        (gen.chain(900), B.default_opts(k=1)),
        (gen.erdos_renyi_paper(20000, 1e-4, gen.SEED_BASE + 4), B.default_opts(schedule_kind=B.SCHED_AUTO, **GPU)),
        (gen.upper_of(gen.random_lower(6000, 0.003, 62)), B.default_opts(triangle=B.UPPER, **GPU)),
    ]


@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("idx", range(6))
def test_multi_rhs_columns_match_oracle(idx, nrhs):
    import torch
    m, opts = _cases()[idx]
    rng = np.random.default_rng(100 * idx + nrhs)
    Bm = rng.uniform(-1.0, 1.0, (m.n, nrhs))
    solve = oracle.solve_upper if m.meta.get("upper") else oracle.solve
    with B.Plan(m, opts) as plan:
        X = plan.solve_multi(torch.from_numpy(Bm).cuda())
        torch.cuda.synchronize()
        assert plan.device_status() == 0
    X = X.cpu().numpy()
    for r in range(nrhs):
        assert oracle.same_bits(X[:, r].copy(), solve(m, Bm[:, r].copy())), (m.name, nrhs, r)


def test_multi_rhs_rejects_overlap():
    import torch
    m = gen.random_lower(500, 0.01, 3)
    with B.Plan(m, B.gpu_opts()) as plan:
        X = torch.zeros(m.n, 3, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError):
            plan.solve_multi(X, X)
