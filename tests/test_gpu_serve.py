"""Serving (continuous batching): requests against resident plans, submitted
while others are on the device, give x bit-identical to the oracle and to the
same request solved alone; the in-flight budget is enforced."""
import time

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    ms = gen.small_set(2500) + [gen.fig_3_1(), gen.chain(200), gen.edgeless(100)]
    opts = [B.gpu_opts()] * len(ms)
    ms += [gen.stencil_2d5(40, 25)]
    opts += [B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)]
    plans = [B.Plan(m, o) for m, o in zip(ms, opts)]
    yield ms, plans
    for p in plans:
        p.close()


def drain(server, pending, timeout=30.0):
    done = {}
    t0 = time.time()
    while len(done) < pending and time.time() - t0 < timeout:
        for tk, ns in server.poll():
            done[tk] = ns
        time.sleep(0.0005)
    return done


@pytest.mark.parametrize("async_exec", [0, 1])
@pytest.mark.parametrize("quantum_us", [50.0, 400.0])
def test_mixed_requests_match_oracle_and_alone(pool, quantum_us, async_exec):
    import torch
    ms, plans = pool
    rng = np.random.default_rng(7)
    reqs = []
    with B.Server(quantum_us=quantum_us, max_slots=16, async_exec=async_exec) as sv:
        for r in range(60):
            i = int(rng.integers(0, len(ms)))
            b = gen.rhs_uniform(ms[i].n, 1000 + r)
            bd = torch.from_numpy(b).cuda()
            xd = torch.full((ms[i].n,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()           # b is written before submit
            tk = sv.submit(plans[i], bd, xd)
            assert tk is not None
            reqs.append((tk, i, b, bd, xd))
            if r % 7 == 0:
                time.sleep(0.001)              # let some complete while others arrive
        done = drain(sv, len(reqs))
        assert len(done) == len(reqs), sv.stats()
        st = sv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
    for tk, i, b, bd, xd in reqs:
        got = xd.cpu().numpy()
        assert oracle.same_bits(got, oracle.solve(ms[i], b)), ms[i].name
        alone = plans[i].solve(bd)
        torch.cuda.synchronize()
        assert oracle.same_bits(got, alone.cpu().numpy())


def test_budget_admission(pool):
    import torch
    ms, plans = pool
    i = 0
    n = ms[i].n
    per_request = 16 * n + 4 * plans[i].info()["supersteps"] + 64
    with B.Server(budget_bytes=2 * per_request + 10, quantum_us=100.0) as sv:
        bd = torch.ones(n, dtype=torch.float64, device="cuda")
        xs = [torch.empty_like(bd) for _ in range(3)]
        torch.cuda.synchronize()
        t1 = sv.submit(plans[i], bd, xs[0])
        t2 = sv.submit(plans[i], bd, xs[1])
        assert t1 is not None and t2 is not None
        deadline = time.time() + 10
        t3 = sv.submit(plans[i], bd, xs[2])
        while t3 is None and time.time() < deadline:   # over budget until one completes
            time.sleep(0.001)
            t3 = sv.submit(plans[i], bd, xs[2])
        assert t3 is not None
        assert len(drain(sv, 3)) == 3
    want = oracle.solve(ms[i], np.ones(n))
    for x in xs:
        assert oracle.same_bits(x.cpu().numpy(), want)


def test_request_larger_than_budget_rejected(pool):
    import torch
    ms, plans = pool
    with B.Server(budget_bytes=64) as sv:
        bd = torch.ones(ms[0].n, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError):
            sv.submit(plans[0], bd, torch.empty_like(bd))


@pytest.mark.parametrize("async_exec", [0, 1])
def test_cancel_queued_and_running_requests(async_exec):
    # one slot: the first request runs while the others wait in the queue; a
    # queued request is withdrawn at once, a running one at the next quantum
    # boundary; withdrawn tickets are never reported, the others stay exact,
    # and the budget and the slot are released
    import torch
    long_m = gen.narrow_band(100_000, 0.03, 42, gen.SEED_BASE + 10)   # thousands of tiny supersteps
    short_m = gen.erdos_renyi(3000, 0.003, gen.SEED_BASE + 44)
    with B.Plan(long_m, B.gpu_opts(schedule_kind=B.SCHED_WAVEFRONT)) as pl, B.Plan(short_m, B.gpu_opts()) as ps:
        want_s = oracle.solve(short_m, np.ones(short_m.n))
        want_l = oracle.solve(long_m, np.ones(long_m.n))
        bl = torch.ones(long_m.n, dtype=torch.float64, device="cuda")
        bs = torch.ones(short_m.n, dtype=torch.float64, device="cuda")
        xs = [torch.full_like(bs, float("nan")) for _ in range(3)]
        xl = [torch.full_like(bl, float("nan")) for _ in range(2)]
        torch.cuda.synchronize()
        with B.Server(quantum_us=100.0, max_slots=1, async_exec=async_exec) as sv:
            t_run = sv.submit(pl, bl, xl[0])          # admitted first, runs for many quanta
            t_q1 = sv.submit(ps, bs, xs[0])           # waits behind it
            t_q2 = sv.submit(ps, bs, xs[1])
            t_q3 = sv.submit(pl, bl, xl[1])
            assert None not in (t_run, t_q1, t_q2, t_q3)
            assert sv.cancel(t_q2)                    # still queued
            assert not sv.cancel(t_q2)                # no longer pending
            time.sleep(0.002)
            assert sv.cancel(t_run)                   # on the device by now (or still queued)
            assert not sv.cancel(987654321)           # unknown ticket
            done = drain(sv, 2)
            assert set(done) == {t_q1, t_q3}, (done, sv.stats())
            t_after = sv.submit(ps, bs, xs[2])        # the slot is usable again
            done.update(drain(sv, 1))
            assert t_after in done and t_run not in done and t_q2 not in done
            st = sv.stats()
            assert st["cancelled"] == 2 and st["completed"] == 3 and st["failed"] == 0, st
            assert st["inflight_bytes"] == 0 and st["queued"] == 0, st
        torch.cuda.synchronize()
        assert oracle.same_bits(xs[0].cpu().numpy(), want_s)
        assert oracle.same_bits(xs[2].cpu().numpy(), want_s)
        assert oracle.same_bits(xl[1].cpu().numpy(), want_l)


@pytest.mark.parametrize("async_exec", [0, 1])
def test_plans_and_vectors_freed_as_their_tickets_complete(async_exec):
    # the server reads nothing of a request after its ticket is polled (or its
    # cancel returned): each plan is destroyed, and its b and x released,
    # the moment its last ticket comes back, while the other requests keep
    # running; their results stay exact
    import torch
    ms = gen.batch_mix(12, seed=gen.SEED_BASE + 1300, lo_exp=2.0, hi_exp=4.5)
    plans = [B.Plan(m, B.gpu_opts() if i % 2 else B.default_opts(schedule_kind=B.SCHED_WAVEFRONT))
             for i, m in enumerate(ms)]
    want = {}
    owner = {}
    left = {i: 0 for i in range(len(ms))}
    with B.Server(quantum_us=60.0, max_slots=8, async_exec=async_exec) as sv:
        for r in range(48):
            i = r % len(ms)
            b = gen.rhs_uniform(ms[i].n, 3000 + r)
            bd = torch.from_numpy(b).cuda()
            xd = torch.full((ms[i].n,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            tk = sv.submit(plans[i], bd, xd)
            assert tk is not None
            want[tk] = (oracle.solve(ms[i], b), xd)
            owner[tk] = i
            left[i] += 1
        del bd, xd
        # withdraw one request on the device, then free its x at once
        victim = next(iter(want))
        if sv.cancel(victim):
            left[owner[victim]] -= 1
            del want[victim]
        t0 = time.time()
        checked = 0
        while want and time.time() - t0 < 60:
            for tk, _ in sv.poll():
                w, xd = want.pop(tk)
                assert oracle.same_bits(xd.cpu().numpy(), w), tk
                checked += 1
                i = owner[tk]
                left[i] -= 1
                if left[i] == 0 and plans[i] is not None:
                    plans[i].close()           # destroyed while the others run
                    plans[i] = None
                del xd
            time.sleep(0.0002)
        assert not want, sv.stats()
        st = sv.stats()
        assert st["failed"] == 0 and st["inflight_bytes"] == 0, st
    for p in plans:
        if p is not None:
            p.close()
    assert checked >= 40
