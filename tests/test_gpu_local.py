"""One-workgroup solve (gltrsv_solve_local): bit-identical to the oracle on
narrow and wide systems, GrowLocal and dealt wavefront schedules, forward
and backward, in place, with IEEE special values, repeated on one plan;
the device layout equals the host-built one."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _opts(kind=B.SCHED_GROWLOCAL, k=64, L=5.0, alpha0=1.0, upper=False):
    return B.default_opts(k=k, L=L, alpha0=alpha0, schedule_kind=kind, exec_hint=2,
                          triangle=B.UPPER if upper else B.LOWER)


MATS = [
    ("fig1_1", lambda: gen.fig_1_1()),
    ("chain", lambda: gen.chain(3000)),
    ("edgeless", lambda: gen.edgeless(10_000)),
    ("nb_03_42", lambda: gen.narrow_band(100_000, 0.03, 42.0, gen.SEED_BASE + 10)),
    ("nb_14_10", lambda: gen.narrow_band(100_000, 0.14, 10.0, gen.SEED_BASE + 10)),
    ("er_1e-4", lambda: gen.erdos_renyi_paper(100_000, 1e-4, gen.SEED_BASE)),
    ("st2d5", lambda: gen.stencil_2d5(200, 150)),
    ("dense_rows", lambda: gen.random_lower(600, 0.2, gen.SEED_BASE + 11)),
]


@pytest.mark.parametrize("name,make", MATS, ids=[m[0] for m in MATS])
@pytest.mark.parametrize("kind", [B.SCHED_GROWLOCAL, B.SCHED_WAVEFRONT, B.SCHED_AUTO], ids=["gl", "wave", "auto"])
def test_local_matches_oracle(name, make, kind):
    import torch
    m = make()
    b = gen.rhs_uniform(m.n, 21)
    want = oracle.solve(m, b)
    print(f"local: {name} kind={kind} n={m.n}", flush=True)
    with B.Plan(m, _opts(kind)) as plan:
        info = plan.info()
        assert info["exec_form"] == B.EXEC_LOCAL and info["local_groups"] > 0
        bd = torch.from_numpy(b).cuda()
        for rep in range(2):
            x = torch.full((m.n,), float("nan"), dtype=torch.float64, device="cuda")
            plan.solve_local(bd, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0, (name, rep)
            assert oracle.same_bits(x.cpu().numpy(), want), (name, kind, rep)
        # solve_auto takes the one-workgroup form; in place
        xi = bd.clone()
        plan.solve_auto(xi, xi)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(xi.cpu().numpy(), want), (name, "in place")


def test_device_layout_equals_host_layout():
    m = gen.narrow_band(30_000, 0.05, 20.0, gen.SEED_BASE + 12)
    with B.Plan(m, _opts()) as plan:
        rec, info = plan.local_records()
        core, sup, _ = plan.schedule()
    hrec, hinfo = B.local_layout(m, core, sup)
    assert np.array_equal(rec, hrec) and np.array_equal(info, hinfo)


def test_backward_and_special_values():
    import torch
    m = gen.upper_of(gen.narrow_band(20_000, 0.05, 20.0, gen.SEED_BASE + 13))
    b = gen.rhs_uniform(m.n, 22)
    b[::97] = -0.0
    b[5::101] = 5e-324
    b[7::211] = np.inf
    b[11::307] = -np.inf
    b[13::401] = np.nan
    want = oracle.solve_upper(m, b)
    with B.Plan(m, _opts(upper=True)) as plan:
        x = plan.solve_local(torch.from_numpy(b).cuda())
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)


def test_paper_parameters_k22():
    import torch
    m = gen.narrow_band(50_000, 0.05, 20.0, gen.SEED_BASE + 14)
    b = gen.rhs_uniform(m.n, 23)
    with B.Plan(m, _opts(k=22, L=500.0, alpha0=20.0)) as plan:
        x = plan.solve_local(torch.from_numpy(b).cuda())
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), oracle.solve(m, b))


def test_tune_includes_local_and_all_forms_agree():
    import torch
    m = gen.narrow_band(100_000, 0.05, 20.0, gen.SEED_BASE + 15)
    b = gen.rhs_uniform(m.n, 24)
    want = oracle.solve(m, b)
    with B.Plan(m, _opts()) as plan:
        bd = torch.from_numpy(b).cuda()
        x = torch.empty_like(bd)
        res = plan.tune(bd, x, reps=3)
        print("tune:", res, flush=True)
        assert set(res["us"]) == {"persistent", "plain", "async", "local"}
        for form in ("solve", "solve_plain", "solve_async", "solve_local"):
            y = getattr(plan, form)(bd)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(y.cpu().numpy(), want), form


def test_plan_without_layout_rejects_local():
    import torch
    m = gen.chain(100)
    with B.Plan(m, B.default_opts()) as plan:
        with pytest.raises(B.GltrsvError):
            plan.solve_local(torch.ones(100, dtype=torch.float64, device="cuda"))
        with pytest.raises(B.GltrsvError):
            plan.set_exec(B.EXEC_LOCAL)
