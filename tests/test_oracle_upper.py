"""Pins of the oracle's backward substitution (the mirror of Eq. (2.1) that
Sec. 2.2 prescribes for upper-triangular systems) and of its schedule.

* Mirror symmetry: renaming every row and column i -> n-1-i turns the upper
  system into a lower one whose rows hold the same entries in the same order,
  so the (separately pinned) forward substitution must produce the reversed
  x bit for bit; a dropped term, a wrong sign or index, or a wrong direction
  in the backward code breaks it.
* Exact cases: integer systems whose every intermediate is an exactly
  representable integer match the rational solution; the bidiagonal system
  with -1 above the diagonal sums b from the right (closed form); a diagonal
  system is a division.
* The schedule of the reverse direction is GrowLocal on the mirrored
  numbering: valid for the upper DAG, and for a DAG without edges it is the
  forward schedule read backwards.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen


def _uppers():
    out = [gen.upper_of(gen.fig_1_1()), gen.upper_of(gen.fig_3_1()), gen.upper_of(gen.chain(40)),
           gen.upper_of(gen.edgeless(7)), gen.upper_of(gen.stencil_2d5(9, 7))]
    for s in range(6):
        out.append(gen.upper_of(gen.random_lower(200, 0.03 + 0.01 * s, 70 + s, band=None if s % 2 else 9)))
    out.append(gen.upper_of(gen.narrow_band(2000, 0.05, 20, 3)))
    return out


@pytest.mark.parametrize("idx", range(12))
def test_mirror_symmetry_with_forward_substitution(idx):
    u = _uppers()[idx]
    b = gen.rhs_uniform(u.n, idx)
    x = oracle.solve_upper(u, b)
    low = oracle.mirror_upper(u, keep_order=True)
    y = oracle.solve(low, b[::-1].copy())
    assert oracle.same_bits(x, y[::-1]), u.name


def test_integer_system_is_exact():
    rng = np.random.default_rng(5)
    n = 60
    rows, cols = [], []
    for i in range(n):
        for j in range(i + 1, min(n, i + 4)):
            if rng.random() < 0.6:
                rows.append(i)
                cols.append(j)
    rp = np.zeros(n + 1, np.int64)
    col, val = [], []
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        col.append(i)
        val.append(1.0)
        A[i][i] = Fraction(1)
        for r, c in zip(rows, cols):
            if r == i:
                a = float(rng.choice([-1, 1]))
                col.append(c)
                val.append(a)
                A[i][c] = Fraction(int(a))
        rp[i + 1] = len(col)
    u = gen.CSR(n, rp, np.array(col, np.int32), np.array(val), "int_upper")
    b = rng.integers(-3, 4, n).astype(np.float64)
    # exact back substitution in rationals
    xe = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        xe[i] = (Fraction(int(b[i])) - sum(A[i][j] * xe[j] for j in range(i + 1, n))) / A[i][i]
    assert all(abs(v) < 2 ** 50 and v.denominator == 1 for v in xe)
    x = oracle.solve_upper(u, b)
    assert [Fraction(v) for v in x] == xe


def test_bidiagonal_closed_form():
    # x_i - x_{i+1} = b_i  =>  x_i = b_i + b_{i+1} + ... + b_{n-1}
    n = 500
    rp = np.zeros(n + 1, np.int64)
    col, val = [], []
    for i in range(n):
        col.append(i)
        val.append(1.0)
        if i + 1 < n:
            col.append(i + 1)
            val.append(-1.0)
        rp[i + 1] = len(col)
    u = gen.CSR(n, rp, np.array(col, np.int32), np.array(val), "bidiag")
    b = np.arange(1, n + 1, dtype=np.float64)
    x = oracle.solve_upper(u, b)
    want = np.array([sum(range(i + 1, n + 1)) for i in range(n)], dtype=np.float64)
    assert np.array_equal(x, want)


def test_diagonal_is_division_and_edge_sizes():
    d = gen.rhs_uniform(300, 1) + 2.5
    b = gen.rhs_uniform(300, 2)
    u = gen.CSR(300, np.arange(301, dtype=np.int64), np.arange(300, dtype=np.int32), d, "diag")
    assert oracle.same_bits(oracle.solve_upper(u, b), b / d)
    e = gen.CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), "empty")
    assert oracle.solve_upper(e, np.zeros(0)).size == 0


def test_upper_layout_is_checked():
    low = gen.fig_1_1()
    with pytest.raises(oracle.OracleError):
        oracle.solve_upper(low, np.ones(low.n))      # diagonal last: not an upper layout


@pytest.mark.parametrize("k,L,a0", [(3, 0.0, 1.0), (22, 500.0, 20.0), (1 << 16, 50.0, 1.0)])
def test_reverse_schedule_is_valid_and_solves_exactly(k, L, a0):
    for u in _uppers():
        pi, sg, S = oracle.growlocal_upper(u, k, L=L, alpha0=a0)
        low = oracle.mirror_upper(u)
        # the schedule of row i is that of vertex n-1-i of the mirrored DAG
        assert oracle.validate(low, k, pi[::-1].copy(), sg[::-1].copy(), S) == oracle.VALID
        # and it respects every edge of the upper DAG directly
        for i in range(u.n):
            for e in range(u.row_ptr[i] + 1, u.row_ptr[i + 1]):
                j = u.col[e]
                assert sg[j] < sg[i] or (sg[j] == sg[i] and pi[j] == pi[i])


def test_reverse_schedule_of_an_edgeless_dag_is_the_forward_one_backwards():
    m = gen.edgeless(1000)
    u = gen.upper_of(m)
    pf, sf, Sf = oracle.growlocal(m, 4, L=500.0)
    pu, su, Su = oracle.growlocal_upper(u, 4, L=500.0)
    assert Su == Sf
    assert np.array_equal(pu, pf[::-1]) and np.array_equal(su, sf[::-1])
    assert not np.array_equal(pu, pf)     # the direction matters


def test_reverse_chain_is_one_superstep_on_one_core():
    u = gen.upper_of(gen.chain(100))
    pi, sg, S = oracle.growlocal_upper(u, 8, L=500.0)
    assert S == 1 and (pi == 0).all()
