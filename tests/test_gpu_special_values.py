"""IEEE special values through every device form, compared with the oracle
bit for bit (NaNs by class, the sign of zero included; the comparison rule of
the oracle's same_bits).

A and b carry signed zeros, subnormals, values whose products overflow to
infinity, infinities, quiet NaNs and the bit pattern 0x7FF4A5A5A5A5A5A5 of
the signalling NaN that the semi-asynchronous forms use as their
"not computed yet" mark.  That mark in the inputs is safe: every kernel runs
with the IEEE mode bit set, and every stored x_i is the result of the
binary64 division sequence, whose last step (v_div_fixup_f64) returns a
quieted NaN whenever an operand is a NaN, so a computed value never carries
the signalling bit pattern and a gathered input equal to it is only ever a
value of b or A, which the kernels never test against the mark.
"""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen

pytestmark = pytest.mark.gpu

MARK = np.array([0x7FF4A5A5A5A5A5A5], dtype=np.uint64).view(np.float64)[0]
OFF_SPECIALS = np.array([0.0, -0.0, 5e-324, -2.5e-310, 1e-300, 1e300, -1e300, 1.7e308, np.inf, -np.inf, np.nan,
                         -np.nan, MARK])
DIAG_SPECIALS = np.array([5e-324, -4e-320, 1e-300, -1e300, 1e308, np.inf, -np.inf, np.nan, MARK, 2.0 ** -1074])
B_SPECIALS = np.array([0.0, -0.0, 5e-324, -1e-310, 1e308, -1e308, np.inf, -np.inf, np.nan, MARK])


def special_system(n, density, seed, frac=0.04):
    """A random lower-triangular matrix with the paper's value distribution,
    a fraction of whose stored values (and of b) is replaced by specials."""
    m = gen.random_lower(n, density, seed)
    rng = np.random.default_rng(seed + 1)
    val = m.val.copy()
    diag = np.zeros(m.nnz, dtype=bool)
    diag[m.row_ptr[1:] - 1] = True
    hit = rng.random(m.nnz) < frac
    off_hit = np.flatnonzero(hit & ~diag)
    val[off_hit] = OFF_SPECIALS[rng.integers(0, OFF_SPECIALS.size, off_hit.size)]
    d_hit = np.flatnonzero(hit & diag)
    val[d_hit] = DIAG_SPECIALS[rng.integers(0, DIAG_SPECIALS.size, d_hit.size)]
    # a few rows with tiny diagonals let the values grow until they overflow
    tiny = np.flatnonzero(diag)[rng.integers(0, n, max(1, n // 50))]
    val[tiny] = 1e-200
    b = gen.rhs_uniform(n, seed + 2)
    bh = rng.random(n) < 0.05
    b[bh] = B_SPECIALS[rng.integers(0, B_SPECIALS.size, int(bh.sum()))]
    return m.with_values(val, name=f"special_n{n}_s{seed}"), b


def _stats(x):
    return {"nan": int(np.isnan(x).sum()), "inf": int(np.isinf(x).sum()),
            "sub": int(((x != 0) & (np.abs(x) < 2.2250738585072014e-308)).sum()),
            "negzero": int(((x == 0) & np.signbit(x)).sum()), "finite": int(np.isfinite(x).sum())}


@pytest.fixture(scope="module")
def cases():
    out = []
    for n, dens, seed, frac in ((3000, 0.002, 11, 0.04), (1500, 0.01, 12, 0.01), (700, 0.05, 13, 0.003)):
        m, b = special_system(n, dens, seed, frac)
        out.append((m, b, oracle.solve(m, b)))
    allx = np.concatenate([c[2] for c in out])
    st = _stats(allx)
    # the inputs really exercise every class
    assert st["nan"] > 0 and st["inf"] > 0 and st["finite"] > 0, st
    return out


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


FORMS = ["solve", "solve_plain", "solve_async"]


@pytest.mark.parametrize("opts_name", ["growlocal", "wavefront", "paper", "wave_cores"])
def test_single_system_forms(cases, opts_name):
    import torch
    opts = {"growlocal": lambda: B.gpu_opts(), "wavefront": lambda: B.default_opts(schedule_kind=B.SCHED_WAVEFRONT),
            "paper": lambda: B.default_opts(), "wave_cores": lambda: B.gpu_opts(core_width=64, k=512)}[opts_name]
    for m, b, want in cases:
        print(f"special values: {m.name} {opts_name}", flush=True)
        with B.Plan(m, opts()) as plan:
            bd = _dev(b)
            for form in FORMS:
                x = torch.full((m.n,), 7.0, dtype=torch.float64, device="cuda")
                getattr(plan, form)(bd, x)
                torch.cuda.synchronize()
                assert plan.device_status() == 0, (m.name, form)
                assert oracle.same_bits(x.cpu().numpy(), want), (m.name, opts_name, form)


def test_multi_rhs_and_in_place(cases):
    import torch
    for m, b, want in cases:
        with B.Plan(m, B.gpu_opts()) as plan:
            cols = np.stack([b, -b, np.where(np.isnan(b), MARK, b[::-1])], axis=1)
            X = plan.solve_multi(_dev(cols))
            torch.cuda.synchronize()
            assert plan.device_status() == 0
            for r in range(cols.shape[1]):
                assert oracle.same_bits(X[:, r].cpu().numpy(), oracle.solve(m, cols[:, r])), (m.name, r)
            for form in FORMS:                  # b aliases x
                xb = _dev(b)
                getattr(plan, form)(xb, xb)
                torch.cuda.synchronize()
                assert oracle.same_bits(xb.cpu().numpy(), want), (m.name, form, "in place")


def test_backward_and_unordered(cases):
    import torch
    for m, b, want in cases:
        u = gen.upper_of(m)
        want_u = oracle.solve_upper(u, b)
        with B.Plan(u, B.gpu_opts(triangle=B.UPPER)) as plan:
            for form in FORMS:
                x = getattr(plan, form)(_dev(b))
                torch.cuda.synchronize()
                assert oracle.same_bits(x.cpu().numpy(), want_u), (m.name, form, "upper")
        with B.Plan(m, B.gpu_opts(reorder=0)) as plan:
            x = plan.solve_unordered(_dev(b))
            torch.cuda.synchronize()
            assert oracle.same_bits(x.cpu().numpy(), want), (m.name, "unordered")


@pytest.mark.parametrize("kind", ["bsp", "async", "wave_async"])
def test_batched_forms(cases, kind):
    import torch
    ms = [c[0] for c in cases]
    opts = B.gpu_opts(core_width=64, k=512) if kind == "wave_async" else B.gpu_opts()
    plans = [B.Plan(m, opts) for m in ms]
    try:
        bs = [_dev(c[1]) for c in cases]
        xs = [torch.full((m.n,), 3.0, dtype=torch.float64, device="cuda") for m in ms]
        with B.Batch(plans, async_exec=kind != "bsp") as bt:
            bt.solve(bs, xs)
            torch.cuda.synchronize()
            assert bt.status() == 0
        for (m, _, want), x in zip(cases, xs):
            assert oracle.same_bits(x.cpu().numpy(), want), (m.name, kind)
    finally:
        for p in plans:
            p.close()


@pytest.mark.parametrize("async_exec", [0, 1])
def test_served(cases, async_exec):
    import time
    import torch
    plans = [B.Plan(c[0], B.gpu_opts()) for c in cases]
    try:
        with B.Server(async_exec=async_exec) as sv:
            want, got = {}, {}
            for p, (m, b, w) in zip(plans, cases):
                x = torch.empty(m.n, dtype=torch.float64, device="cuda")
                t = sv.submit(p, _dev(b), x)
                want[t], got[t] = w, x
            t0 = time.time()
            done = set()
            while len(done) < len(want) and time.time() - t0 < 30:
                done.update(t for t, _ in sv.poll())
                time.sleep(0.001)
            assert done == set(want)
            for t in want:
                assert oracle.same_bits(got[t].cpu().numpy(), want[t])
    finally:
        for p in plans:
            p.close()
