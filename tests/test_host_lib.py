"""Host side of the HIP library, on the CPU: the shared library loads and
exports every function include/gltrsv.h declares; CSR checks return the
documented codes; the library's wavefronts, GrowLocal schedule and Sec. 5
order equal the oracle's bit for bit (two independent implementations)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gltrsv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gltrsv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in B.SIGNATURES, f"{name} has no binding"


def test_version_and_defaults():
    assert B.load().gltrsv_version().decode().count(".") == 2
    o = B.default_opts()
    assert (o.k, o.L, o.alpha0, o.growth, o.accept) == (22, 500.0, 20.0, 1.5, 0.97)
    assert o.schedule_kind == B.SCHED_GROWLOCAL


def _csr(n, rp, col, val):
    return gen.CSR(n, np.asarray(rp, np.int64), np.asarray(col, np.int32), np.asarray(val, np.float64))


@pytest.mark.parametrize("case,code", [
    (lambda: _csr(2, [0, 1, 3], [0, 1, 1], [1.0, 2.0, 1.0]), -4),      # duplicate column
    (lambda: _csr(2, [0, 2, 3], [0, 1, 1], [1.0, 2.0, 1.0]), -2),      # above the diagonal
    (lambda: _csr(2, [0, 1, 2], [0, 0], [1.0, 1.0]), -3),              # row 1 lacks its diagonal
    (lambda: _csr(2, [0, 1, 2], [0, 1], [1.0, 0.0]), -3),              # zero diagonal
    (lambda: _csr(2, [0, 1, 2], [0, 5], [1.0, 1.0]), -5),              # column out of range
    (lambda: _csr(2, [0, 1, 3], [0, 1, 0], [1.0, 1.0, 1.0]), -4),      # columns fall
])
def test_check_csr_codes(case, code):
    assert B.check_csr(case()) == code


def test_bad_options_rejected():
    m = gen.fig_1_1()
    for bad in (dict(k=0), dict(alpha0=0.5), dict(growth=1.0), dict(L=-1.0), dict(schedule_kind=7),
                dict(analysis_threads=-1), dict(pack=9), dict(blocks=-2), dict(funnel_max_weight=-1),
                dict(exec_hint=3), dict(exec_hint=-1), dict(exec_hint=2, k=65), dict(exec_hint=2, core_width=64),
                dict(reorder=2), dict(reorder=-1), dict(triangle=5), dict(core_width=32)):
        with pytest.raises(B.GltrsvError):
            B.schedule(m, B.default_opts(**bad))


def cases():
    out = [gen.fig_1_1(), gen.fig_3_1(), gen.edgeless(1000), gen.chain(300), gen.stencil_2d5(25, 9),
           gen.random_lower(1, 0.5, 1)]
    for s in range(12):
        out.append(gen.random_lower(150, 0.02 + 0.02 * (s % 4), 40 + s, band=None if s % 2 else 5))
    out += gen.small_set(3000)
    return out


PARAMS = [dict(), dict(k=1), dict(k=3, L=0.0), dict(k=4096, L=50.0, alpha0=1.0),
          dict(k=100, L=10.0, alpha0=2.0, growth=2.0, accept=0.9), dict(k=1 << 16, L=5.0, alpha0=1.0)]


@pytest.mark.parametrize("pidx", range(len(PARAMS)))
def test_growlocal_equals_oracle(pidx):
    p = PARAMS[pidx]
    for m in cases():
        o = B.default_opts(**p)
        core, sup, S = B.schedule(m, o)
        pi, sg, S2 = oracle.growlocal(m, o.k, L=o.L, alpha0=o.alpha0, growth=o.growth, theta=o.accept)
        assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg), m.name


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_growlocal_workers_do_not_change_the_schedule(threads):
    # the iterations of a superstep run on several host threads; the
    # acceptance rule reads them in order, so the schedule is the oracle's
    for p in (PARAMS[0], PARAMS[3], PARAMS[4], PARAMS[5]):
        for m in cases()[:8] + [gen.random_lower(3000, 0.003, 77)]:
            o = B.default_opts(analysis_threads=threads, **p)
            core, sup, S = B.schedule(m, o)
            pi, sg, S2 = oracle.growlocal(m, o.k, L=o.L, alpha0=o.alpha0, growth=o.growth, theta=o.accept)
            assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg), (m.name, threads)


@pytest.mark.parametrize("nblocks", [2, 5, 16])
def test_block_parallel_growlocal_equals_oracle(nblocks):
    for p in (PARAMS[0], PARAMS[2], PARAMS[3]):
        for m in cases()[:10]:
            o = B.default_opts(blocks=nblocks, **p)
            core, sup, S = B.schedule(m, o)
            pi, sg, S2 = oracle.growlocal_blocks(m, o.k, nblocks, L=o.L, alpha0=o.alpha0, growth=o.growth,
                                                 theta=o.accept)
            assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg), (m.name, nblocks)


def test_block_parallel_growlocal_threads_equal_oracle():
    # 3e5 rows: the blocks are scheduled on several host threads
    m = gen.erdos_renyi(300_000, 1e-5, gen.SEED_BASE + 9)
    o = B.gpu_opts(blocks=8)
    core, sup, S = B.schedule(m, o)
    pi, sg, S2 = oracle.growlocal_blocks(m, o.k, 8, L=o.L, alpha0=o.alpha0, growth=o.growth, theta=o.accept)
    assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)


def test_levels_wavefront_and_order_equal_oracle():
    for m in cases():
        lv, nl = B.levels(m)
        lv2, nl2 = oracle.levels(m)
        assert nl == nl2 and np.array_equal(lv, lv2)
        core, sup, S = B.schedule(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT))
        pi, sg, S2 = oracle.wavefront_schedule(m)
        assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)
        core, sup, S = B.schedule(m, B.gpu_opts())
        perm = B.reorder(core, sup)
        perm2, _ = oracle.reorder(m, core, sup)
        assert np.array_equal(perm, perm2)
        assert oracle.validate(m, 1 << 16, core, sup, S) == oracle.VALID


def test_empty_matrix():
    m = gen.CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert B.check_csr(m) == 0
    core, sup, S = B.schedule(m)
    assert S == 0


def test_auto_schedule_avoids_serial_grid_and_stays_valid():
    grid = gen.stencil_2d5(60)
    _, _, S_gl = B.schedule(grid, B.gpu_opts())
    core, sup, S = B.schedule(grid, B.gpu_opts(schedule_kind=B.SCHED_AUTO))
    _, nl = oracle.levels(grid)
    assert S_gl == 1 and S == nl                      # wavefront chosen for the one-source grid
    assert oracle.validate(grid, int(core.max()) + 1, core, sup, S) == oracle.VALID
    for m in cases():
        core, sup, S = B.schedule(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO))
        k = int(core.max()) + 1 if m.n else 1
        assert oracle.validate(m, k, core, sup, S) == oracle.VALID, m.name
        g = B.schedule(m, B.gpu_opts())
        w = B.schedule(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT))
        assert (np.array_equal(core, g[0]) and np.array_equal(sup, g[1])) or \
               (np.array_equal(core, w[0]) and np.array_equal(sup, w[1]))


def _uppers():
    out = [gen.upper_of(m) for m in (gen.fig_1_1(), gen.fig_3_1(), gen.chain(300), gen.edgeless(500),
                                      gen.stencil_2d5(25, 9))]
    for s in range(6):
        out.append(gen.upper_of(gen.random_lower(150, 0.02 + 0.02 * (s % 4), 40 + s, band=None if s % 2 else 5)))
    out.append(gen.upper_of(gen.narrow_band(3000, 0.05, 20, 2)))
    return out


@pytest.mark.parametrize("pidx", [0, 2, 3, 4])
def test_upper_growlocal_equals_oracle(pidx):
    p = PARAMS[pidx]
    for u in _uppers():
        for nb in (1, 3):
            o = B.default_opts(triangle=B.UPPER, blocks=nb, **p)
            core, sup, S = B.schedule(u, o)
            pi, sg, S2 = oracle.growlocal_upper(u, o.k, L=o.L, alpha0=o.alpha0, growth=o.growth, theta=o.accept,
                                                nblocks=nb)
            assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg), (u.name, nb)


def test_upper_wavefront_and_layout_checks():
    for u in _uppers():
        core, sup, S = B.schedule(u, B.default_opts(triangle=B.UPPER, schedule_kind=B.SCHED_WAVEFRONT))
        pi, sg, S2 = oracle.wavefront_schedule(oracle.mirror_upper(u))
        assert S == S2 and np.array_equal(core, pi[::-1]) and np.array_equal(sup, sg[::-1])
    low = gen.random_lower(50, 0.1, 3)
    with pytest.raises(B.GltrsvError) as e:
        B.schedule(low, B.default_opts(triangle=B.UPPER))
    assert e.value.code == -2                      # entries below the diagonal
    with pytest.raises(B.GltrsvError) as e:
        B.schedule(gen.upper_of(low), B.default_opts())
    assert e.value.code == -2                      # entries above the diagonal
    with pytest.raises(B.GltrsvError):
        B.schedule(low, B.default_opts(triangle=5))


@pytest.mark.parametrize("cap", [1, 6, 30, 400])
def test_funnel_growlocal_equals_oracle(cap):
    for p in (PARAMS[0], PARAMS[2], PARAMS[3]):
        for m in cases()[:12]:
            o = B.default_opts(funnel_max_weight=cap, **p)
            core, sup, S = B.schedule(m, o)
            pi, sg, S2, part = oracle.funnel_growlocal(m, o.k, cap, L=o.L, alpha0=o.alpha0, growth=o.growth,
                                                       theta=o.accept)
            assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg), (m.name, cap)


def test_funnel_upper_equals_oracle_on_the_mirror():
    for u in _uppers()[:8]:
        o = B.default_opts(triangle=B.UPPER, funnel_max_weight=25, **PARAMS[3])
        core, sup, S = B.schedule(u, o)
        pi, sg, S2, _ = oracle.funnel_growlocal(oracle.mirror_upper(u), o.k, 25, L=o.L, alpha0=o.alpha0,
                                                growth=o.growth, theta=o.accept)
        assert S == S2 and np.array_equal(core, pi[::-1]) and np.array_equal(sup, sg[::-1]), u.name


def test_given_schedule_is_checked_against_definition_2_1():
    # rejected before any device work, so this runs on the CPU
    m = gen.random_lower(300, 0.02, 7)
    core, sup, S = B.schedule(m, B.gpu_opts())
    bad_edge = np.zeros(m.n, np.int32), np.zeros(m.n, np.int32)
    bad_edge[0][:] = np.arange(m.n)                     # one superstep, every row on its own core
    bad_range = core.copy(), sup.copy()
    bad_range[0][5] = -1
    for sched in (bad_edge, bad_range):
        with pytest.raises(B.GltrsvError) as e:
            B.Plan(m, B.gpu_opts(), schedule=sched)
        assert e.value.code == -1 and "given schedule" in str(e.value)
