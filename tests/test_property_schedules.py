"""Property tests (CPU): on many random small DAGs the library's schedulers
give exactly the oracle's schedules -- GrowLocal (Algorithm 3.1), its
block-parallel form (Sec. 3.1), Funnel + GrowLocal (Sec. 4) and the reverse
direction for upper-triangular systems -- and every schedule is valid
(Definition 2.1).  Hypothesis draws the pattern and the parameters and shrinks
any failure to a minimal case."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2503_05408_amd import binding as B
from paper_2503_05408_amd import gen


@st.composite
def lower_patterns(draw):
    n = draw(st.integers(1, 36))
    density = draw(st.sampled_from([0.0, 0.05, 0.15, 0.35, 0.7]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    band = draw(st.sampled_from([None, 2, 6]))
    return gen.random_lower(n, density, seed, band=band)


params = st.fixed_dictionaries({
    "k": st.sampled_from([1, 2, 3, 7, 64, 1 << 16]),
    "L": st.sampled_from([0.0, 3.0, 50.0, 500.0]),
    "alpha0": st.sampled_from([1.0, 2.0, 20.0]),
    "growth": st.sampled_from([1.5, 2.0]),
    "accept": st.sampled_from([0.9, 0.97, 1.0]),
})

# 10,000 random cases in all (4,000 for plain GrowLocal, 2,000 for each variant)
SETTINGS = settings(max_examples=2000, deadline=None, suppress_health_check=[HealthCheck.too_slow])
SETTINGS_MAIN = settings(max_examples=4000, deadline=None, suppress_health_check=[HealthCheck.too_slow])


def _oracle_args(p):
    return dict(L=p["L"], alpha0=p["alpha0"], growth=p["growth"], theta=p["accept"])


@SETTINGS_MAIN
@given(lower_patterns(), params)
def test_growlocal_library_equals_oracle(m, p):
    core, sup, S = B.schedule(m, B.default_opts(**p))
    pi, sg, S2 = oracle.growlocal(m, p["k"], **_oracle_args(p))
    assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)
    assert oracle.validate(m, p["k"], pi, sg, S2) == oracle.VALID


@SETTINGS
@given(lower_patterns(), params, st.integers(2, 9))
def test_block_parallel_library_equals_oracle(m, p, nblocks):
    core, sup, S = B.schedule(m, B.default_opts(blocks=nblocks, **p))
    pi, sg, S2 = oracle.growlocal_blocks(m, p["k"], nblocks, **_oracle_args(p))
    assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)
    assert oracle.validate(m, p["k"], pi, sg, S2) == oracle.VALID


@SETTINGS
@given(lower_patterns(), params, st.sampled_from([1, 3, 8, 40, 10 ** 6]))
def test_funnel_library_equals_oracle(m, p, cap):
    core, sup, S = B.schedule(m, B.default_opts(funnel_max_weight=cap, **p))
    pi, sg, S2, _ = oracle.funnel_growlocal(m, p["k"], cap, **_oracle_args(p))
    assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)
    assert oracle.validate(m, p["k"], pi, sg, S2) == oracle.VALID


@SETTINGS
@given(lower_patterns(), params)
def test_upper_library_equals_oracle(m, p):
    u = gen.upper_of(m)
    core, sup, S = B.schedule(u, B.default_opts(triangle=B.UPPER, **p))
    pi, sg, S2 = oracle.growlocal_upper(u, p["k"], **_oracle_args(p))
    assert S == S2 and np.array_equal(core, pi) and np.array_equal(sup, sg)
