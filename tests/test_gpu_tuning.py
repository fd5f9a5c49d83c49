"""Execution forms and their autotuner (GPU): gltrsv_solve_auto runs the
preferred form, gltrsv_plan_set_exec sets it, gltrsv_plan_tune measures the
three forms and keeps the fastest; every form stays bit-identical to the
oracle, the JSON tables of tuning.tune_cached and tuning.best_plan (schedule
and form) reproduce a stored choice."""
import json

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen, tuning

pytestmark = pytest.mark.gpu

MATRICES = [
    ("er", lambda: gen.erdos_renyi(4000, 0.003, gen.SEED_BASE + 41), B.gpu_opts()),
    ("grid", lambda: gen.stencil_3d7(24), B.gpu_opts(schedule_kind=B.SCHED_AUTO)),
    ("upper", lambda: gen.upper_of(gen.narrow_band(3000, 0.1, 12, gen.SEED_BASE + 42)),
     B.gpu_opts(triangle=B.UPPER)),
]


def _want(m, b):
    return oracle.solve_upper(m, b) if m.meta.get("upper") else oracle.solve(m, b)


@pytest.mark.parametrize("case", [c[0] for c in MATRICES])
def test_tune_picks_the_fastest_form_and_every_form_is_exact(case):
    import torch
    _, make, opts = next(c for c in MATRICES if c[0] == case)
    m = make()
    b = gen.rhs_uniform(m.n, 5)
    want = _want(m, b)
    bd = torch.from_numpy(b).cuda()
    with B.Plan(m, opts) as plan:
        assert plan.info()["exec_form"] == B.EXEC_PERSISTENT
        x = torch.full_like(bd, float("nan"))
        res = plan.tune(bd, x, reps=3)
        torch.cuda.synchronize()
        print(case, res, flush=True)
        assert set(res["us"]) == {"persistent", "plain", "async"}
        assert all(v > 0 for v in res["us"].values())
        assert res["form"] == min(res["us"], key=res["us"].get)
        assert B.EXEC_NAMES[plan.info()["exec_form"]] == res["form"]
        assert oracle.same_bits(x.cpu().numpy(), want)            # x holds the solution
        for form in (B.EXEC_PERSISTENT, B.EXEC_PLAIN, B.EXEC_ASYNC):
            plan.set_exec(form)
            assert plan.info()["exec_form"] == form
            x.fill_(float("nan"))
            plan.solve_auto(bd, x)
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), form
            y = bd.clone()                                        # in place: b aliases x
            plan.solve_auto(y, y)
            torch.cuda.synchronize()
            assert oracle.same_bits(y.cpu().numpy(), want), ("in place", form)


def test_exec_hint_sets_the_initial_form_and_bad_arguments_are_rejected():
    import torch
    m = gen.erdos_renyi(1500, 0.004, gen.SEED_BASE + 43)
    with B.Plan(m, B.gpu_opts(exec_hint=1)) as plan:
        assert plan.info()["exec_form"] == B.EXEC_ASYNC
        with pytest.raises(B.GltrsvError):
            plan.set_exec(3)
        with pytest.raises(B.GltrsvError):
            plan.set_exec(-1)
        b = torch.ones(m.n, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError):
            plan.tune(b, b)                                        # overlapping b and x
        big = torch.ones(2 * m.n, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError):
            plan.tune(big[: m.n], big[m.n // 2: m.n // 2 + m.n])   # partial overlap
        with pytest.raises(B.GltrsvError):
            plan.tune(b, torch.empty_like(b), reps=0)
        assert plan.info()["exec_form"] == B.EXEC_ASYNC           # unchanged by the rejected calls


def test_tune_reports_a_forced_timeout_and_keeps_the_preference():
    # a spin limit of one poll (forced from the host): the measured solves end
    # early with the error word set, every wave leaves normally, tune returns
    # ETIMEDOUT and leaves the preferred form as it was
    import torch
    m = gen.stencil_3d7(40)
    with B.Plan(m, B.default_opts(schedule_kind=B.SCHED_WAVEFRONT)) as plan:
        plan.set_exec(B.EXEC_PLAIN)
        plan.set_spin_limit(1)
        b = torch.ones(m.n, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GltrsvError) as ei:
            plan.tune(b, torch.empty_like(b), reps=1)
        assert ei.value.code == -9
        assert plan.info()["exec_form"] == B.EXEC_PLAIN
        assert plan.device_status() == 0
        plan.set_spin_limit(5_000_000)
        x = plan.solve_auto(b)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), oracle.solve(m, np.ones(m.n)))


def test_tuning_table_round_trip(tmp_path):
    import torch
    path = str(tmp_path / "tuning.json")
    m = gen.stencil_2d5(60, 50)
    want = oracle.solve(m, np.ones(m.n))
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) as plan:
        form = tuning.tune_cached(plan, path, reps=2)
        key = tuning.tuning_key(plan)
    table = json.load(open(path))
    assert table[key]["form"] == form
    # a stored choice is applied without measuring: plant another form
    other = "plain" if form != "plain" else "async"
    table[key]["form"] = other
    tuning.store_table(path, table)
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) as plan:
        assert tuning.tuning_key(plan) == key
        assert tuning.tune_cached(plan, path) == other
        assert B.EXEC_NAMES[plan.info()["exec_form"]] == other
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
    # a different schedule of the same pattern has its own entry
    with B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_GROWLOCAL, k=7)) as plan:
        assert tuning.tuning_key(plan) != key


def test_best_plan_over_schedules_and_forms(tmp_path):
    import torch
    path = str(tmp_path / "best.json")
    m = gen.erdos_renyi(20000, 2e-4, gen.SEED_BASE + 45)
    want = oracle.solve(m, np.ones(m.n))
    plan, entry = tuning.best_plan(m, B.gpu_opts(), path, reps=3)
    print(entry, flush=True)
    with plan:
        assert len(entry["us"]) == 6 and entry["core_width"] == 1
        fastest = min(entry["us"], key=entry["us"].get)
        assert fastest == f"{entry['label']}/{entry['form']}"
        kind = {"growlocal": B.SCHED_GROWLOCAL, "wavefront": B.SCHED_WAVEFRONT}[entry["schedule"]]
        assert plan.info()["schedule_kind"] == kind
        assert B.EXEC_NAMES[plan.info()["exec_form"]] == entry["form"]
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
    # from the table: only the stored choice is built, nothing is measured
    table = tuning.load_table(path)
    (key,) = table
    table[key] = {"schedule": "wavefront", "form": "plain", "us": {}}
    tuning.store_table(path, table)
    plan, entry = tuning.best_plan(m, B.gpu_opts(), path)
    with plan:
        assert entry["schedule"] == "wavefront" and entry["form"] == "plain"
        assert plan.info()["schedule_kind"] == B.SCHED_WAVEFRONT
        assert plan.info()["exec_form"] == B.EXEC_PLAIN
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
    # other schedule parameters are another entry
    assert not key.startswith(tuning.matrix_key(m, B.gpu_opts(L=20.0)))


def test_best_plan_with_wave_cores(tmp_path):
    import torch
    m = gen.erdos_renyi(4000, 0.03, gen.SEED_BASE + 46)    # rows of ~60 entries
    want = oracle.solve(m, np.ones(m.n))
    plan, entry = tuning.best_plan(m, B.gpu_opts(k=1024), str(tmp_path / "w.json"), reps=2, core_widths=(1, 64))
    print(entry, flush=True)
    with plan:
        assert len(entry["us"]) == 12               # 2 schedules x 2 widths x 3 forms
        fastest = min(entry["us"], key=entry["us"].get)
        assert fastest == f"{entry['label']}/{entry['form']}"
        assert plan.info()["core_width"] == entry["core_width"]
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)


def test_best_plan_over_schedule_parameters_and_one_workgroup(tmp_path):
    # GrowLocal at several (k, L) (the paper's L is architecture-dependent,
    # Sec. 3) and the one-workgroup form beside the device-wide ones
    import torch
    path = str(tmp_path / "kl.json")
    m = gen.narrow_band(20_000, 0.05, 20.0, gen.SEED_BASE + 49)
    want = oracle.solve(m, np.ones(m.n))
    params = [(1 << 16, 50.0), (4096, 50.0), (1 << 16, 10.0)]
    plan, entry = tuning.best_plan(m, B.gpu_opts(), path, reps=2, params=params, local=True)
    print(entry, flush=True)
    with plan:
        # 1 wavefront + 3 GrowLocal candidates x 3 forms, 2 one-workgroup candidates x 4 forms
        assert len(entry["us"]) == 4 * 3 + 2 * 4
        fastest = min(entry["us"], key=entry["us"].get)
        assert fastest == f"{entry['label']}/{entry['form']}"
        if entry["schedule"] == "growlocal":
            assert (entry["k"], entry["L"]) in params + [(64, 5.0)]
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)
    # the stored choice, (k, L) and execution hint included, is rebuilt as is
    table = tuning.load_table(path)
    (key,) = table
    table[key] = {"schedule": "growlocal", "core_width": 1, "k": 4096, "L": 50.0, "exec_hint": 0,
                  "form": "persistent", "us": {}}
    tuning.store_table(path, table)
    plan, entry = tuning.best_plan(m, B.gpu_opts(), path, params=params, local=True)
    with plan:
        assert plan.opts.k == 4096 and plan.info()["exec_form"] == B.EXEC_PERSISTENT
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert oracle.same_bits(x.cpu().numpy(), want)
    table[key] = {"schedule": "wavefront", "core_width": 1, "k": None, "L": None, "exec_hint": 2,
                  "form": "local", "us": {}}
    tuning.store_table(path, table)
    plan, entry = tuning.best_plan(m, B.gpu_opts(), path, params=params, local=True)
    with plan:
        assert plan.info()["exec_form"] == B.EXEC_LOCAL and plan.info()["local_groups"] > 0
        x = plan.solve_auto(torch.ones(m.n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert oracle.same_bits(x.cpu().numpy(), want)


def test_best_batch_picks_the_fastest_configuration(tmp_path):
    import torch
    ms = [gen.erdos_renyi(3000, 0.003, gen.SEED_BASE + 47), gen.stencil_2d5(40, 30),
          gen.narrow_band(2500, 0.05, 20, gen.SEED_BASE + 48), gen.chain(200)]
    plans = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO)) for m in ms]
    plans_a = [B.Plan(m, B.gpu_opts(schedule_kind=B.SCHED_AUTO, exec_hint=1)) for m in ms]
    bs = [torch.from_numpy(gen.rhs_uniform(m.n, 20 + i)).cuda() for i, m in enumerate(ms)]
    wants = [oracle.solve(m, b.cpu().numpy()) for m, b in zip(ms, bs)]
    xs = [torch.full_like(b, float("nan")) for b in bs]
    path = str(tmp_path / "batch.json")
    bt, entry = tuning.best_batch(plans, bs, xs, plans_async=plans_a, claims=(1, 2), reps=2, path=path)
    print(entry, flush=True)
    with bt:
        assert len(entry["ms"]) == 4
        assert f"{entry['form']}/{entry['per_claim']}" == min(entry["ms"], key=entry["ms"].get)
        for x in xs:
            x.fill_(float("nan"))
        bt.solve(bs, xs)
        torch.cuda.synchronize()
        assert bt.status() == 0
        for x, w in zip(xs, wants):
            assert oracle.same_bits(x.cpu().numpy(), w)
    # a stored choice is used as it is
    table = tuning.load_table(path)
    (key,) = table
    table[key] = {"form": "bsp", "per_claim": 2, "ms": {}}
    tuning.store_table(path, table)
    bt, entry = tuning.best_batch(plans, bs, xs, plans_async=plans_a, path=path)
    with bt:
        assert entry["form"] == "bsp" and entry["per_claim"] == 2
        assert bt.info()["systems"] == len(ms)
    for p in plans + plans_a:
        p.close()
