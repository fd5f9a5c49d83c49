"""Device packing (the reorder of Sec. 5 plus the lane-interleaved stream,
filled by row-length, LDS-staged wavefront prefix-scan and scatter kernels)
gives the same stream as the host packer, byte for byte, and its plans solve
bit-exactly against the oracle.  Sizes span several scan tiles (2048 rows
each) and, for the largest case, several tiles of tile totals."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

GPU = dict(k=1 << 16, L=50.0, alpha0=1.0)


def _streams_equal(m, opts):
    with B.Plan(m, B.default_opts(pack=B.PACK_HOST, **opts)) as ph, \
            B.Plan(m, B.default_opts(pack=B.PACK_DEVICE, **opts)) as pd:
        ih, idv = ph.info(), pd.info()
        assert ih["device_packed"] == 0 and idv["device_packed"] == 1
        assert ih["stream_slots"] == idv["stream_slots"] and ih["chunks"] == idv["chunks"]
        wh, vh = ph.stream()
        wd, vd = pd.stream()
    assert np.array_equal(wh, wd), m.name
    assert np.array_equal(vh.view(np.uint64), vd.view(np.uint64)), m.name
    return ih


@pytest.mark.parametrize("maker,opts", [
    (lambda: gen.fig_1_1(), dict()),
    (lambda: gen.fig_3_1(), dict(k=2, L=0.0)),
    (lambda: gen.edgeless(1), dict()),
    (lambda: gen.edgeless(5000), GPU),
    (lambda: gen.chain(3000), dict(k=1)),
    (lambda: gen.chain(3000), dict(schedule_kind=B.SCHED_WAVEFRONT)),
    (lambda: gen.stencil_2d5(70, 61), GPU),
    (lambda: gen.stencil_3d7(20), dict(schedule_kind=B.SCHED_WAVEFRONT)),
    (lambda: gen.random_lower(9000, 0.002, 21), GPU),
    (lambda: gen.random_lower(9000, 0.002, 21), dict(k=7, L=10.0)),
    (lambda: gen.narrow_band(20000, 0.05, 20, 4), GPU),
    (lambda: gen.erdos_renyi_paper(30000, 1e-4, gen.SEED_BASE + 7), dict(schedule_kind=B.SCHED_AUTO, **GPU)),
])
def test_device_stream_equals_host_stream(maker, opts):
    m = maker()
    info = _streams_equal(m, opts)
    print(m.name, info["supersteps"], info["chunks"], info["stream_slots"], flush=True)


def test_device_packed_plan_solves_exactly():
    import torch
    for m, opts in [(gen.random_lower(9000, 0.002, 22), GPU), (gen.narrow_band(20000, 0.03, 42, 5), GPU),
                    (gen.stencil_2d5(90), dict(schedule_kind=B.SCHED_WAVEFRONT))]:
        b = gen.rhs_uniform(m.n, 3)
        want = oracle.solve(m, b)
        with B.Plan(m, B.default_opts(pack=B.PACK_DEVICE, **opts)) as plan:
            x = plan.solve(torch.from_numpy(b).cuda())
            xp = plan.solve_plain(torch.from_numpy(b).cuda())
            torch.cuda.synchronize()
            assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want), m.name
        assert oracle.same_bits(xp.cpu().numpy(), want), m.name


def test_device_packing_many_scan_tiles():
    # 5e6 rows: 2442 scan tiles, so the tile totals need two passes of the
    # single-workgroup scan
    m = gen.erdos_renyi(5_000_000, 4e-7, gen.SEED_BASE + 11)
    info = _streams_equal(m, dict(schedule_kind=B.SCHED_WAVEFRONT))
    assert info["n"] == 5_000_000
