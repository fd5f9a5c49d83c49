"""Host analysis under sanitizers (CPU): the library's analysis code
(analysis.cpp: CSR checks, GrowLocal with its worker pool, block-parallel
and Funnel scheduling, the wavefront schedule, the Definition 2.1 check, the
Sec. 5 order and the stream packing) is compiled with g++ together with
tests/sanitize_analysis.cpp, once with AddressSanitizer +
UndefinedBehaviorSanitizer and once with ThreadSanitizer, and run on lower-
and upper-triangular inputs and on malformed copies.  Any sanitizer report
fails the run (halt_on_error).  The GrowLocal schedule that the sanitized
build writes must equal the oracle's (Algorithm 3.1)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_05408_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize_analysis.cpp")

FLAVOURS = {
    "address,undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "thread": ["-fsanitize=thread"],
}
ENV = {
    "address,undefined": {"ASAN_OPTIONS": "halt_on_error=1:detect_leaks=1",
                          "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
    "thread": {"TSAN_OPTIONS": "halt_on_error=1"},
}


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = {}
    d = tmp_path_factory.mktemp("sanitize")
    for name, flags in FLAVOURS.items():
        exe = str(d / ("driver_" + name.replace(",", "_")))
        cmd = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer", *flags,
               "-I", CSRC, "-I", os.path.join(ROOT, "include"), DRIVER, os.path.join(CSRC, "analysis.cpp"),
               "-o", exe, "-pthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
            pytest.skip(f"{name} runtime not installed")
        assert r.returncode == 0, r.stderr[-3000:]
        out[name] = exe
    return out


def _write(m, path, upper):
    with open(path, "wb") as f:
        np.array([m.n, m.nnz], dtype=np.int64).tofile(f)
        np.array([1 if upper else 0], dtype=np.int32).tofile(f)
        m.row_ptr.astype(np.int64).tofile(f)
        m.col.astype(np.int32).tofile(f)
        m.val.astype(np.float64).tofile(f)


def _run(exe, flavour, m, tmp_path, upper=False, threads=4):
    mp, sp = str(tmp_path / "m.bin"), str(tmp_path / "s.bin")
    _write(m, mp, upper)
    env = dict(os.environ, **ENV[flavour])
    r = subprocess.run([exe, mp, sp, str(threads)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr, \
        r.stderr[-4000:]
    s = np.fromfile(sp, dtype=np.int32)
    return s[:m.n], s[m.n:]


CASES = [
    ("er", lambda: gen.erdos_renyi(3000, 0.004, gen.SEED_BASE + 31)),
    ("nb", lambda: gen.narrow_band(3000, 0.1, 12, gen.SEED_BASE + 32)),
    ("grid", lambda: gen.stencil_2d5(40, 30)),
    ("chain", lambda: gen.chain(500)),
    ("fig1_1", lambda: gen.fig_1_1()),
]


@pytest.mark.parametrize("flavour", list(FLAVOURS))
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_analysis_clean_and_equal_to_oracle(binaries, flavour, case, tmp_path):
    m = dict(CASES)[case]()
    core, sup = _run(binaries[flavour], flavour, m, tmp_path)
    pi, sg, _ = oracle.growlocal(m, 4, L=10.0, alpha0=1.0)
    assert np.array_equal(core, pi) and np.array_equal(sup, sg)


@pytest.mark.parametrize("flavour", list(FLAVOURS))
def test_upper_analysis_clean_and_equal_to_oracle(binaries, flavour, tmp_path):
    u = gen.upper_of(gen.erdos_renyi(2000, 0.005, gen.SEED_BASE + 33))
    core, sup = _run(binaries[flavour], flavour, u, tmp_path, upper=True)
    pi, sg, _ = oracle.growlocal_upper(u, 4, L=10.0, alpha0=1.0)
    assert np.array_equal(core, pi) and np.array_equal(sup, sg)


def test_worker_pool_under_thread_sanitizer_larger(binaries, tmp_path):
    """More rows and eight workers, so the pool's trial and commit phases
    interleave many times."""
    m = gen.erdos_renyi(20000, 0.0006, gen.SEED_BASE + 34)
    core, sup = _run(binaries["thread"], "thread", m, tmp_path, threads=8)
    pi, sg, _ = oracle.growlocal(m, 4, L=10.0, alpha0=1.0)
    assert np.array_equal(core, pi) and np.array_equal(sup, sg)
