"""Per-wave record streams of the semi-asynchronous wave-core solve, built on
the host (gltrsv_wave_streams): every row once, as a header with its
diagonal followed by its off-diagonals in stored order (Eq. (2.1)'s order),
tasks in the order of Sec. 5 dealt to the waves round robin, and run task
by task they give the oracle's x bit for bit under every valid schedule
(Definition 2.1)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

HDR, INTL, MASK, PAD = 0x80000000, 0x40000000, 0x3FFFFFFF, 0xFFFFFFFF
RING = 64


def _schedule(m, kind, upper=False, **kw):
    opts = B.default_opts(schedule_kind=kind, triangle=B.UPPER if upper else B.LOWER, **kw)
    core, sup, _ = B.schedule(m, opts)
    return core, sup


def _task_span(st, k, waves):
    """First and one-past-last slot of task k's records."""
    tasks = len(st["stask"])
    end = st["stask"][k + waves] if k + waves < tasks else st["sbeg"][k % waves + 1] - 1
    return int(st["stask"][k]), int(end)


def _run(st, n, b, waves):
    """Executes the tasks in their global order, each from its own span: a
    row's entries read x, or the ring for one of the task's recent rows."""
    x = np.full(n, np.nan)
    done = np.zeros(n, dtype=bool)
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        _run_tasks(st, b, waves, x, done)
    return x


def _run_tasks(st, b, waves, x, done):
    scol, sval = st["scol"], st["sval"]
    for k in range(len(st["stask"])):
        o, end = _task_span(st, k, waves)
        assert scol[o] & HDR and scol[o] & INTL and scol[o] != PAD, "a task starts with a task-first header"
        ring = []
        while o < end:
            w = int(scol[o])
            assert w & HDR and w != PAD
            row, diag = w & MASK, sval[o]
            acc = b[row]
            o += 1
            while o < end and not (int(scol[o]) & HDR):
                c = int(scol[o])
                if c & INTL:
                    d = c & MASK
                    assert 0 < d < RING and d <= len(ring)
                    g = ring[-d]
                else:
                    assert done[c], "a column read from memory was computed by an earlier task"
                    g = x[c]
                acc = acc - sval[o] * g
                o += 1
            x[row] = acc / diag
            done[row] = True
            ring.append(x[row])


CASES = [
    ("fig1_1", gen.fig_1_1),
    ("chain", lambda: gen.chain(400)),
    ("edgeless", lambda: gen.edgeless(300)),
    ("dense_rows", lambda: gen.erdos_renyi(600, 0.12, gen.SEED_BASE + 71)),   # rows over 64 entries
    ("nb", lambda: gen.narrow_band(3000, 0.05, 20.0, gen.SEED_BASE + 72)),
    ("st2d5", lambda: gen.stencil_2d5(40, 30)),
]
SCHEDS = [
    ("growlocal_k4", dict(kind=B.SCHED_GROWLOCAL, k=4)),
    ("growlocal_k64", dict(kind=B.SCHED_GROWLOCAL, k=64, L=50.0, alpha0=1.0)),
    ("wavefront", dict(kind=B.SCHED_WAVEFRONT)),
]


@pytest.mark.parametrize("case", [c[0] for c in CASES])
@pytest.mark.parametrize("sched", [s[0] for s in SCHEDS])
@pytest.mark.parametrize("waves", [1, 3, 64])
def test_streams_run_to_the_oracle(case, sched, waves):
    m = dict(CASES)[case]()
    kw = dict(dict(SCHEDS)[sched])
    core, sup = _schedule(m, kw.pop("kind"), **kw)
    st = B.wave_streams(m, core, sup, waves)
    b = gen.rhs_uniform(m.n, 5)
    assert oracle.same_bits(_run(st, m.n, b, waves), oracle.solve(m, b))


def test_layout_of_the_streams():
    m = gen.narrow_band(2000, 0.05, 20.0, gen.SEED_BASE + 73)
    core, sup = _schedule(m, B.SCHED_GROWLOCAL, k=8)
    waves = 5
    st = B.wave_streams(m, core, sup, waves)
    scol, sval, sbeg, stask = st["scol"], st["sval"], st["sbeg"], st["stask"]
    # tasks: runs of one core in a superstep; their number and order
    order = np.lexsort((np.arange(m.n), core, sup))
    runs = 1 + int(np.count_nonzero((np.diff(sup[order]) != 0) | (np.diff(core[order]) != 0)))
    assert len(stask) == runs
    # slot v holds tasks v, v + W, ... in that order, then one PAD; padding after
    for v in range(waves):
        ks = list(range(v, len(stask), waves))
        starts = [int(stask[k]) for k in ks]
        assert starts == sorted(starts)
        if ks:
            assert starts[0] == sbeg[v]
        assert scol[sbeg[v + 1] - 1] == PAD
    assert np.all(scol[sbeg[-1]:] == PAD) and np.all(sval[sbeg[-1]:] == 0.0)
    assert len(scol) - sbeg[-1] >= 128
    # every row once as a header with its diagonal, then its off-diagonals
    # in stored order (columns, or ring distances within the task)
    hdr = (scol & HDR) != 0
    hdr &= scol != PAD
    rows = (scol[hdr] & MASK).astype(np.int64)
    assert np.array_equal(np.sort(rows), np.arange(m.n))
    pos = np.flatnonzero(hdr)
    for p, r in zip(pos, rows):
        a, e = m.row_ptr[r], m.row_ptr[r + 1]
        assert sval[p] == m.val[e - 1]
        ent = scol[p + 1:p + 1 + (e - 1 - a)]
        assert not np.any(ent & HDR)
        np.testing.assert_array_equal(sval[p + 1:p + 1 + (e - 1 - a)], m.val[a:e - 1])
        plain = (ent & INTL) == 0
        np.testing.assert_array_equal(ent[plain], m.col[a:e - 1][plain])


def test_backward_substitution_streams():
    m = gen.upper_of(gen.narrow_band(2500, 0.05, 20.0, gen.SEED_BASE + 74))
    core, sup = _schedule(m, B.SCHED_GROWLOCAL, upper=True, k=16)
    st = B.wave_streams(m, core, sup, 7, triangle=B.UPPER)
    b = gen.rhs_uniform(m.n, 6)
    assert oracle.same_bits(_run(st, m.n, b, 7), oracle.solve_upper(m, b))


def test_special_values_pass_through_the_streams():
    m = gen.narrow_band(1500, 0.05, 20.0, gen.SEED_BASE + 75)
    b = gen.rhs_uniform(m.n, 7)
    b[::97] = -0.0
    b[5::101] = 5e-324
    b[7::211] = np.inf
    b[13::401] = np.nan
    core, sup = _schedule(m, B.SCHED_WAVEFRONT)
    st = B.wave_streams(m, core, sup, 9)
    assert oracle.same_bits(_run(st, m.n, b, 9), oracle.solve(m, b))


def test_bad_arguments():
    m = gen.chain(50)
    core = np.zeros(m.n, np.int32)
    sup = np.arange(m.n, dtype=np.int32)
    with pytest.raises(B.GltrsvError):
        B.wave_streams(m, core, sup, 0)
    with pytest.raises(B.GltrsvError):   # dependent rows on two cores in one superstep
        B.wave_streams(m, (np.arange(m.n) % 2).astype(np.int32), np.zeros(m.n, np.int32), 3)
    empty = gen.edgeless(0)
    st = B.wave_streams(empty, np.zeros(0, np.int32), np.zeros(0, np.int32), 4)
    assert len(st["stask"]) == 0 and list(st["sbeg"]) == [0, 1, 2, 3, 4]


def _run_waves(st, n, b, waves):
    """Runs the streams the way the semi-asynchronous kernel does, without
    its global order: every wave walks only its own stream and takes a row
    once every column it reads from memory has been computed; the waves take
    turns.  The run must finish (a wave's next row always becomes ready:
    Definition 2.1 and the task order) and give the oracle's bits."""
    scol, sval, sbeg = st["scol"], st["sval"], st["sbeg"]
    x = np.full(n, np.nan)
    done = np.zeros(n, dtype=bool)
    pos = [int(sbeg[v]) for v in range(waves)]
    end = [int(sbeg[v + 1]) - 1 for v in range(waves)]
    rings = [[] for _ in range(waves)]
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        while True:
            moved = False
            for v in range(waves):
                if pos[v] >= end[v]:
                    continue
                o = pos[v]
                w = int(scol[o])
                assert w & HDR and w != PAD
                e = o + 1
                while e < end[v] and not (int(scol[e]) & HDR):
                    e += 1
                cols = [int(c) for c in scol[o + 1:e] if not (int(c) & INTL)]
                if not all(done[c] for c in cols):
                    continue
                if w & INTL:
                    rings[v] = []
                row, acc = w & MASK, b[w & MASK]
                for k in range(o + 1, e):
                    c = int(scol[k])
                    g = rings[v][-(c & MASK)] if c & INTL else x[c]
                    acc = acc - sval[k] * g
                x[row] = acc / sval[o]
                done[row] = True
                rings[v].append(x[row])
                pos[v] = e
                moved = True
            if all(pos[v] >= end[v] for v in range(waves)):
                return x
            assert moved, "no wave can take its next row"


@st.composite
def _small_systems(draw):
    n = draw(st.integers(1, 40))
    density = draw(st.sampled_from([0.0, 0.05, 0.2, 0.5]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    band = draw(st.sampled_from([None, 3, 8]))
    return gen.random_lower(n, density, seed, band=band)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(_small_systems(), st.sampled_from([1, 2, 3, 5, 64, 300]),
       st.sampled_from([("growlocal", 1), ("growlocal", 3), ("growlocal", 64), ("wavefront", 0)]),
       st.integers(0, 2 ** 31 - 1), st.booleans())
def test_streams_run_by_waves_of_their_own(m, waves, sched, bseed, upper):
    kind, k = sched
    if upper:
        m = gen.upper_of(m)
    core, sup = (_schedule(m, B.SCHED_WAVEFRONT, upper=upper) if kind == "wavefront"
                 else _schedule(m, B.SCHED_GROWLOCAL, upper=upper, k=k, L=3.0, alpha0=1.0))
    s = B.wave_streams(m, core, sup, waves, triangle=B.UPPER if upper else B.LOWER)
    b = gen.rhs_uniform(m.n, bseed % 1000)
    want = oracle.solve_upper(m, b) if upper else oracle.solve(m, b)
    assert oracle.same_bits(_run(s, m.n, b, waves), want)
    assert oracle.same_bits(_run_waves(s, m.n, b, waves), want)
