"""GPU measurement probes of the library: the copy kernel copies exactly,
and the gather probe (the solve's traffic without its dependencies) returns,
for x = ones, exactly the left-to-right sum of each row's off-diagonals --
a plain definition checked here with a Python loop."""
import numpy as np
import pytest

from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _row_sums_in_order(m):
    out = np.zeros(m.n)
    for i in range(m.n):
        s = 0.0
        for e in range(m.row_ptr[i], m.row_ptr[i + 1] - 1):
            s += float(m.val[e])
        out[i] = s
    return out


def test_copy_probe_copies_exactly():
    import torch
    src = torch.from_numpy(gen.rhs_uniform(1 << 16, 5)).cuda()
    dst = torch.full_like(src, float("nan"))
    B.copy_probe(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("maker,opts", [
    (lambda: gen.random_lower(3000, 0.004, 11), dict(k=1 << 16, L=50.0, alpha0=1.0)),
    (lambda: gen.random_lower(3000, 0.004, 11), dict()),
    (lambda: gen.stencil_2d5(40), dict(k=1 << 16, L=50.0, alpha0=1.0)),
    (lambda: gen.chain(500), dict(k=3, L=0.0)),
    (lambda: gen.edgeless(300), dict()),
    (lambda: gen.narrow_band(5000, 0.05, 20, 3), dict(schedule_kind=B.SCHED_WAVEFRONT)),
])
def test_gather_probe_row_sums(maker, opts):
    import torch
    m = maker()
    with B.Plan(m, B.default_opts(**opts)) as plan:
        x = torch.ones(m.n, dtype=torch.float64, device="cuda")
        y = torch.full_like(x, float("nan"))
        plan.gather_probe(x, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
    want = _row_sums_in_order(m)
    assert np.array_equal(got.view(np.int64), want.view(np.int64)), m.name
