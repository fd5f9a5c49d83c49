"""Performance floors (GPU): loose lower bounds on the throughput of the
n = 1e7 Erdos-Renyi workload, about half of what this device measures, so
that a regression that doubles the solve time fails while run-to-run noise
does not.  Every timed result is also checked against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu


def _ms(fn, b, x, reps=10):
    import torch
    fn(b, x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn(b, x)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def test_er_1e7_throughput_floor():
    import torch
    n = 10_000_000
    m = gen.erdos_renyi(n, 20.0 / (n - 1), gen.SEED_BASE + 200)
    want = oracle.solve(m, np.ones(n))
    with B.Plan(m, B.gpu_opts()) as plan:
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        x = torch.empty_like(b)
        floor_ms = _ms(plan.gather_probe, torch.ones_like(b), x, reps=5)
        for name, fn, min_rows_s in (("persistent", plan.solve, 2.2e9), ("async", plan.solve_async, 2.5e9),
                                     ("plain", plan.solve_plain, 2.0e9)):
            ms = _ms(fn, b, x)
            assert plan.device_status() == 0
            assert oracle.same_bits(x.cpu().numpy(), want), name
            rows_s = n / (ms * 1e-3)
            print(f"{name}: {ms:.3f} ms, {rows_s:.3e} rows/s, gather floor {floor_ms:.3f} ms", flush=True)
            assert rows_s >= min_rows_s, (name, rows_s)
            assert ms <= 2.0 * floor_ms, (name, ms, floor_ms)
