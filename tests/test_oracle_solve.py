"""Pins of the oracle's forward substitution (Eq. (2.1)) to things other than
itself: exact integer/dyadic solutions, the IEEE definition of each binary64
operation (exact rational result, then rounding), closed forms for diagonal
matrices, and the backward-error bound of triangular solves.

Each pin is chosen so that a plausible mistake fails it: a dropped term, a
wrong sign or a wrong index changes exact solutions; a fused
multiply-add, a reassociated sum or a reciprocal-multiply changes the
rounding, and the inputs are checked to tell those variants apart.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen


def rows(m):
    for i in range(m.n):
        lo, hi = int(m.row_ptr[i]), int(m.row_ptr[i + 1])
        yield i, [(int(m.col[e]), float(m.val[e])) for e in range(lo, hi - 1)], float(m.val[hi - 1])


def exact_solution(m, b):
    """Forward substitution in exact rational arithmetic."""
    x = []
    for i, offs, d in rows(m):
        acc = Fraction(b[i])
        for j, a in offs:
            acc -= Fraction(a) * x[j]
        x.append(acc / Fraction(d))
    return x


def rnd(q: Fraction) -> float:
    """Round an exact rational to the nearest binary64 (ties to even);
    CPython's int/int true division is correctly rounded."""
    return q.numerator / q.denominator


def rounded_solution(m, b, variant="running"):
    """Eq. (2.1) with every operation's exact result rounded to binary64.

    variant "running": acc <- rnd(acc - rnd(a*x)) in stored order, then
    rnd(acc / d) -- the reading the oracle implements.  The others model
    plausible mistakes: "fma" (product not rounded), "sum_first" (sum the
    products, then subtract), "reciprocal" (multiply by rnd(1/d))."""
    x = []
    for i, offs, d in rows(m):
        if variant == "sum_first":
            s = Fraction(0)
            for j, a in offs:
                s = Fraction(rnd(s + Fraction(rnd(Fraction(a) * Fraction(x[j])))))
            acc = Fraction(rnd(Fraction(b[i]) - s))
        else:
            acc = Fraction(b[i])
            for j, a in offs:
                prod = Fraction(a) * Fraction(x[j])
                if variant != "fma":
                    prod = Fraction(rnd(prod))
                acc = Fraction(rnd(acc - prod))
        if variant == "reciprocal":
            x.append(rnd(acc * Fraction(rnd(1 / Fraction(d)))))
        else:
            x.append(rnd(acc / Fraction(d)))
    return np.array(x)


# --------------------------------------------------------------------------
# P1: exact solutions
# --------------------------------------------------------------------------

def _exactly_representable_run(m, b):
    """True if every intermediate of the running subtraction is an exactly
    representable binary64 (so no rounding happens in any order)."""
    x = []
    for i, offs, d in rows(m):
        acc = Fraction(b[i])
        for j, a in offs:
            p = Fraction(a) * x[j]
            if Fraction(rnd(p)) != p:
                return False
            acc -= p
            if Fraction(rnd(acc)) != acc:
                return False
        xi = acc / Fraction(d)
        if Fraction(rnd(xi)) != xi:
            return False
        x.append(xi)
    return True


@pytest.mark.parametrize("seed", range(12))
def test_integer_unit_diagonal_exact(seed):
    m = gen.random_lower(40, 0.08, 1000 + seed, values="int_unit")
    b = gen.rhs_int(m.n, 2000 + seed)
    assert _exactly_representable_run(m, b)
    want = exact_solution(m, b)
    assert all(q.denominator == 1 for q in want)
    got = oracle.solve(m, b)
    assert [Fraction(v) for v in got] == want


@pytest.mark.parametrize("seed", range(12))
def test_dyadic_diagonal_exact(seed):
    """Diagonals +-2^e keep the exact solution dyadic."""
    m = gen.random_lower(30, 0.06, 3000 + seed, values="int_pow2")
    b = gen.rhs_int(m.n, 4000 + seed)
    if not _exactly_representable_run(m, b):
        pytest.skip("an intermediate needs more than 53 bits for this seed")
    got = oracle.solve(m, b)
    assert [Fraction(v) for v in got] == exact_solution(m, b)


def test_exact_pins_catch_plausible_mistakes():
    """The integer inputs above distinguish a dropped term, a sign flip and a
    wrong index (the column shifted by one)."""
    m = gen.random_lower(40, 0.08, 1000, values="int_unit")
    b = gen.rhs_int(m.n, 2000)
    good = exact_solution(m, b)
    # dropped last term of each row
    bad = []
    for i, offs, d in rows(m):
        acc = Fraction(b[i])
        for j, a in offs[:-1]:
            acc -= Fraction(a) * bad[j]
        bad.append(acc / Fraction(d))
    assert bad != good
    # sign flip
    bad = []
    for i, offs, d in rows(m):
        acc = Fraction(b[i])
        for j, a in offs:
            acc += Fraction(a) * bad[j]
        bad.append(acc / Fraction(d))
    assert bad != good
    # wrong index: x_{j-1} instead of x_j
    bad = []
    for i, offs, d in rows(m):
        acc = Fraction(b[i])
        for j, a in offs:
            acc -= Fraction(a) * bad[max(j - 1, 0)]
        bad.append(acc / Fraction(d))
    assert bad != good


def test_fig_1_1_integer_example():
    """The 6x6 pattern of Fig. 1.1 with off-diagonals -1 and unit diagonal:
    x_a = b_a, x_b = b_b + x_a, x_c = b_c + x_b, x_d = b_d + x_b,
    x_e = b_e + x_c, x_f = b_f + x_d."""
    m = gen.fig_1_1()
    b = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    want = [1, 3, 6, 7, 11, 13]
    assert oracle.solve(m, b).tolist() == want


# --------------------------------------------------------------------------
# rounding: each operation rounded on its own, in the stated order
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_rounding_matches_ieee_definition(seed):
    m = gen.random_lower(60, 0.15, 5000 + seed, values="paper")
    b = gen.rhs_uniform(m.n, 6000 + seed)
    want = rounded_solution(m, b, "running")
    got = oracle.solve(m, b)
    assert oracle.same_bits(got, want)


def test_rounding_inputs_separate_the_variants():
    """The inputs of the rounding pin are sensitive: the fused, sum-first and
    reciprocal variants each give different bits somewhere."""
    seen = {"fma": False, "sum_first": False, "reciprocal": False}
    for seed in range(6):
        m = gen.random_lower(60, 0.15, 5000 + seed, values="paper")
        b = gen.rhs_uniform(m.n, 6000 + seed)
        ref = rounded_solution(m, b, "running")
        for v in seen:
            if not oracle.same_bits(rounded_solution(m, b, v), ref):
                seen[v] = True
    assert all(seen.values()), seen


# --------------------------------------------------------------------------
# P2: diagonal matrices
# --------------------------------------------------------------------------

def test_diagonal_matrix_is_one_division():
    rng = np.random.default_rng(7)
    n = 4000
    d = rng.uniform(0.5, 2.0, n) * np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0)
    m = gen.edgeless(n).with_values(np.ascontiguousarray(d))
    b = rng.uniform(-1.0, 1.0, n)
    got = oracle.solve(m, b)
    assert oracle.same_bits(got, b / d)
    # the inputs would expose a reciprocal-multiply
    assert not oracle.same_bits(b * (1.0 / d), b / d)


def test_special_values():
    """Signed zeros and infinities follow IEEE division and subtraction."""
    m = gen.edgeless(4).with_values(np.array([1.0, -1.0, 2.0, 0.5]))
    b = np.array([0.0, 0.0, np.inf, -np.inf])
    got = oracle.solve(m, b)
    want = np.array([0.0, -0.0, np.inf, -np.inf])
    assert oracle.same_bits(got, want)
    assert np.signbit(got[1])


# --------------------------------------------------------------------------
# P4: backward error of a triangular solve
# --------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [lambda: gen.stencil_2d5(40), lambda: gen.stencil_3d7(11),
                                   lambda: gen.random_lower(400, 0.05, 77, values="paper"),
                                   lambda: gen.narrow_band(800, 0.14, 10.0, 78)],
                         ids=["st2d5", "st3d7", "er400", "nb800"])
def test_backward_error_bound(maker):
    """Componentwise: |b - A x|_i <= gamma_m * (|A| |x|)_i with m the stored
    entries of row i and gamma_m = m u / (1 - m u), u = 2^-53 (standard bound
    for substitution); the residual is formed exactly."""
    m = maker()
    b = gen.rhs_uniform(m.n, 11)
    x = oracle.solve(m, b)
    u = 2.0 ** -53
    for i in range(m.n):
        lo, hi = int(m.row_ptr[i]), int(m.row_ptr[i + 1])
        r = Fraction(b[i])
        s = Fraction(0)
        for e in range(lo, hi):
            t = Fraction(float(m.val[e])) * Fraction(float(x[m.col[e]]))
            r -= t
            s += abs(t)
        k = hi - lo
        gamma = Fraction(k) * Fraction(u) / (1 - Fraction(k) * Fraction(u))
        assert abs(r) <= gamma * s, i


def test_same_bits_rule():
    a = np.array([0.0, np.nan, 1.0])
    assert oracle.same_bits(a, np.array([0.0, -np.nan, 1.0]))
    assert not oracle.same_bits(a, np.array([-0.0, np.nan, 1.0]))
    assert not oracle.same_bits(a, np.array([0.0, 1.0, 1.0]))
    assert not oracle.same_bits(a, np.array([0.0, np.nan, math.nextafter(1.0, 2.0)]))


def test_rejects_malformed():
    m = gen.fig_1_1()
    bad = m.with_values(m.val.copy())
    bad.val[-1] = 0.0
    with pytest.raises(oracle.OracleError):
        oracle.solve(bad, np.ones(6))
    r = gen.random_lower(50, 0.3, 3)
    i = next(i for i in range(r.n) if r.row_ptr[i + 1] - r.row_ptr[i] >= 3)
    col = r.col.copy()
    a = r.row_ptr[i]
    col[a], col[a + 1] = col[a + 1], col[a]          # two off-diagonals out of order
    assert oracle.check_csr(gen.CSR(r.n, r.row_ptr, col, r.val)) != 0
    col = r.col.copy()
    col[a] = i + 1 if i + 1 < r.n else i             # above or on the diagonal
    assert oracle.check_csr(gen.CSR(r.n, r.row_ptr, col, r.val)) != 0
