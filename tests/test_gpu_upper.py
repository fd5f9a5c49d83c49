"""Backward substitution on the GPU (upper-triangular systems, the mirror of
Eq. (2.1), Sec. 2.2): every solve form against the oracle bit for bit, host
and device packing of the same stream, and a batch mixing forward and
backward systems."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

GPU = dict(k=1 << 16, L=50.0, alpha0=1.0)
OPTS = {"paper": dict(), "gpu": GPU, "wavefront": dict(schedule_kind=B.SCHED_WAVEFRONT),
        "auto": dict(schedule_kind=B.SCHED_AUTO, **GPU), "blocks": dict(blocks=4, **GPU)}


def _uppers():
    return [gen.upper_of(gen.fig_1_1()), gen.upper_of(gen.chain(700)), gen.upper_of(gen.edgeless(130)),
            gen.upper_of(gen.stencil_2d5(60, 45)), gen.upper_of(gen.stencil_3d7(14)),
            gen.upper_of(gen.random_lower(8000, 0.002, 51)), gen.upper_of(gen.narrow_band(20000, 0.05, 20, 9)),
            gen.upper_of(gen.erdos_renyi_paper(20000, 1e-4, gen.SEED_BASE + 3))]


@pytest.mark.parametrize("optname", list(OPTS))
@pytest.mark.parametrize("idx", range(8))
def test_backward_solves_match_oracle(idx, optname):
    import torch
    u = _uppers()[idx]
    b = gen.rhs_uniform(u.n, idx)
    want = oracle.solve_upper(u, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(u, B.default_opts(triangle=B.UPPER, **OPTS[optname])) as plan:
        x1 = plan.solve(bd)
        x2 = plan.solve_plain(bd)
        x3 = plan.solve_async(bd)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        core, sup, perm = plan.schedule()
        S = plan.info()["supersteps"]
    print(u.name, optname, S, flush=True)
    for x in (x1, x2, x3):
        assert oracle.same_bits(x.cpu().numpy(), want), (u.name, optname)
    # the plan's schedule is a valid schedule of the upper DAG (per row)
    for i in range(u.n):
        for e in range(u.row_ptr[i] + 1, u.row_ptr[i + 1]):
            j = u.col[e]
            assert sup[j] < sup[i] or (sup[j] == sup[i] and core[j] == core[i])


@pytest.mark.parametrize("idx", [3, 5, 6, 7])
def test_backward_device_stream_equals_host_stream(idx):
    u = _uppers()[idx]
    with B.Plan(u, B.default_opts(triangle=B.UPPER, pack=B.PACK_HOST, **GPU)) as ph, \
            B.Plan(u, B.default_opts(triangle=B.UPPER, pack=B.PACK_DEVICE, **GPU)) as pd:
        wh, vh = ph.stream()
        wd, vd = pd.stream()
    assert np.array_equal(wh, wd) and np.array_equal(vh.view(np.uint64), vd.view(np.uint64))


def test_batch_mixing_forward_and_backward_systems():
    import torch
    lows = [gen.random_lower(5000, 0.002, 81), gen.narrow_band(9000, 0.03, 42, 2), gen.stencil_2d5(50)]
    systems = lows + [gen.upper_of(m) for m in lows]
    plans = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO, triangle=B.UPPER if m.meta.get("upper") else B.LOWER))
             for m in systems]
    bs = [torch.from_numpy(gen.rhs_uniform(m.n, i)).cuda() for i, m in enumerate(systems)]
    xs = [torch.empty_like(b) for b in bs]
    B.solve_batched(plans, bs, xs)
    torch.cuda.synchronize()
    for i, m in enumerate(systems):
        b = bs[i].cpu().numpy()
        want = oracle.solve_upper(m, b) if m.meta.get("upper") else oracle.solve(m, b)
        assert oracle.same_bits(xs[i].cpu().numpy(), want), m.name
    for p in plans:
        p.close()
