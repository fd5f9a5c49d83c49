"""Pins of the Funnel coarsening oracle (Sec. 4):

* the approximate transitive reduction removes exactly the long edges of
  triangles (checked against boolean matrix products) and keeps every
  reachability (transitive closures are equal);
* every part is an in-funnel (Definition 4.4): a cascade (Definition 4.2,
  checked by brute-force reachability) with at most one vertex that has an
  outgoing cut edge;
* the coarsened graph is acyclic (Proposition 4.3) and the root numbering is
  a topological order of it;
* every in-tree is an in-funnel, so an in-tree collapses into one part
  without a weight cap; with a cap of one weight unit every part is a
  single vertex;
* Funnel + GrowLocal pulled back to the rows is a valid schedule of the
  original DAG and executes to the serial solve bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen


def _adj(m):
    a = np.zeros((m.n, m.n), dtype=bool)
    for i in range(m.n):
        for e in range(m.row_ptr[i], m.row_ptr[i + 1] - 1):
            a[m.col[e], i] = True          # edge (j, i)
    return a


def _closure(a):
    r = a.copy()
    n = len(a)
    for k in range(n):
        r |= np.outer(r[:, k], r[k, :])
    return r


def _mats():
    out = [gen.fig_1_1(), gen.fig_3_1(), gen.chain(30), gen.stencil_2d5(7, 6)]
    for s in range(5):
        out.append(gen.random_lower(70, 0.04 + 0.03 * s, 90 + s, band=None if s % 2 else 8))
    return out


@pytest.mark.parametrize("idx", range(9))
def test_transitive_reduction_removes_long_triangle_edges_only(idx):
    m = _mats()[idx]
    a = _adj(m)
    two = (a.astype(np.int64) @ a.astype(np.int64)) > 0
    kept = oracle.transitive_reduction(m)
    k = np.zeros_like(a)
    for w, ps in enumerate(kept):
        for u in ps:
            k[u, w] = True
    assert np.array_equal(k, a & ~two)
    assert np.array_equal(_closure(k), _closure(a))


def _reduced_adj(m):
    kept = oracle.transitive_reduction(m)
    a = np.zeros((m.n, m.n), dtype=bool)
    for w, ps in enumerate(kept):
        for u in ps:
            a[u, w] = True
    return a


@pytest.mark.parametrize("cap", [1, 5, 12, 40, 10 ** 9])
@pytest.mark.parametrize("idx", range(9))
def test_parts_are_in_funnels_and_the_coarse_graph_is_acyclic(idx, cap):
    m = _mats()[idx]
    part = oracle.funnel_partition(m, cap)
    a = _reduced_adj(m)
    reach = _closure(a) | np.eye(m.n, dtype=bool)
    weight = np.diff(m.row_ptr)
    for q in range(int(part.max()) + 1):
        U = np.flatnonzero(part == q)
        inside = np.zeros(m.n, dtype=bool)
        inside[U] = True
        out_cut = [u for u in U if (a[u] & ~inside).any()]
        in_cut = [v for v in U if (a[:, v] & ~inside).any()]
        assert len(out_cut) <= 1
        for v in in_cut:
            for u in out_cut:
                assert reach[v, u]                       # cascade
        assert len(U) == 1 or weight[U].sum() <= cap
    cm, cw = oracle.coarse_dag(m, part)                  # asserts the root order is topological
    assert cw.sum() == weight.sum()
    # Proposition 4.3 directly: the coarse graph has no cycle
    ca = _adj(cm)
    assert not (_closure(ca) & np.eye(cm.n, dtype=bool)).any()


def test_in_tree_is_one_part_and_cap_one_gives_singletons():
    rng = np.random.default_rng(3)
    n = 200
    child = [int(rng.integers(v + 1, n)) for v in range(n - 1)]
    entries = [(child[v] + 1, v + 1) for v in range(n - 1)]     # 1-based (row, col)
    m = gen.from_entries(n, entries)
    part = oracle.funnel_partition(m, 10 ** 9)
    assert (part == 0).all()
    part1 = oracle.funnel_partition(m, 1)
    assert int(part1.max()) + 1 == n


@pytest.mark.parametrize("cap", [4, 20, 200])
@pytest.mark.parametrize("k,L,a0", [(3, 0.0, 1.0), (22, 500.0, 20.0), (1 << 16, 50.0, 1.0)])
def test_funnel_growlocal_schedule_is_valid_and_exact(cap, k, L, a0):
    for s in range(4):
        m = gen.random_lower(250, 0.02 + 0.01 * s, 120 + s, band=None if s % 2 else 15)
        pi, sg, S, part = oracle.funnel_growlocal(m, k, cap, L=L, alpha0=a0)
        assert oracle.validate(m, k, pi, sg, S) == oracle.VALID
        # rows of one part share core and superstep
        for q in range(int(part.max()) + 1):
            U = part == q
            assert len(set(pi[U])) == 1 and len(set(sg[U])) == 1
        b = gen.rhs_uniform(m.n, s)
        assert oracle.same_bits(oracle.bsp_solve(m, b, pi, sg), oracle.solve(m, b))
