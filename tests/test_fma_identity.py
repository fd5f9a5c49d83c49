"""The wave-core kernels' DPP row subtraction adds each product to the
running sum as fma(p, -1, acc).  The product by -1 is exact, so the fused
operation rounds once, as the subtraction acc - p of Eq. (2.1) does: the
bits are those of acc - p for every pair of binary64 values, signed zeros,
subnormals, infinities and overflow included (NaN results stay NaN).  This
checks that reading with the C library's correctly rounded fma on the host."""
import ctypes
import ctypes.util

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def fma():
    path = ctypes.util.find_library("m")
    if path is None:
        pytest.skip("libm not found")
    lib = ctypes.CDLL(path)
    lib.fma.restype = ctypes.c_double
    lib.fma.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    return lib.fma


SPECIALS = np.array([0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, -1e-310, 1.0, -1.0, 1.5, 1e300,
                     -1e300, 1.7976931348623157e308, -1.7976931348623157e308, np.inf, -np.inf, np.nan])


def test_fma_by_minus_one_is_the_subtraction(fma):
    rng = np.random.default_rng(2503054)
    # random magnitudes over the whole exponent range, and near-cancelling pairs
    a = rng.uniform(-1, 1, 4000) * 2.0 ** rng.integers(-1074, 1024, 4000)
    p = rng.uniform(-1, 1, 4000) * 2.0 ** rng.integers(-1074, 1024, 4000)
    near = a[:1000] * (1 + rng.uniform(-1e-15, 1e-15, 1000))
    acc = np.concatenate([a, a[:1000], np.repeat(SPECIALS, SPECIALS.size)])
    prod = np.concatenate([p, near, np.tile(SPECIALS, SPECIALS.size)])
    with np.errstate(over="ignore", invalid="ignore"):
        want = acc - prod
    got = np.array([fma(float(q), -1.0, float(c)) for c, q in zip(acc, prod)])
    assert oracle.same_bits(got, want)


def test_a_plain_fused_product_differs(fma):
    # control: fusing the product itself (fma(v, g, -acc)) skips its rounding
    # and does change bits, which is why only the exact product by -1 is fused
    rng = np.random.default_rng(7)
    v, g, acc = rng.uniform(-2, 2, 2000), rng.uniform(-2, 2, 2000), rng.uniform(-2, 2, 2000)
    fused = np.array([-fma(float(x), float(y), -float(c)) for x, y, c in zip(v, g, acc)])
    assert not oracle.same_bits(fused, acc - v * g)
