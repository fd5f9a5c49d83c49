"""Pins of the oracle's wavefronts, GrowLocal (Algorithm 3.1), validator
(Definition 2.1), reordering (Sec. 5) and BSP execution.

GrowLocal is a heuristic, so its pins are: the worked figures, closed forms
derived by hand from the rules (edgeless DAGs, chains, the exclusivity and
blocking rules on small constructions), an independent model of the rules on
edgeless DAGs across many parameters, and the invariants every schedule must
satisfy.
"""
import json
import math
import os
from collections import deque

import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def counts_per_superstep(pi, sigma, S, k):
    return [np.bincount(pi[sigma == s], minlength=k).tolist() for s in range(S)]


# --------------------------------------------------------------------------
# worked figures
# --------------------------------------------------------------------------

def test_fig_1_1_dag_and_wavefronts():
    g = load_golden("fig1_1.json")
    m = gen.from_entries(g["n"], g["nonzeros_1based"])
    lab = g["labels"]
    edges = sorted((lab[int(m.col[e])], lab[i]) for i in range(m.n)
                   for e in range(m.row_ptr[i], m.row_ptr[i + 1] - 1))
    assert edges == sorted(tuple(e) for e in g["dag_edges"])
    lv, nl = oracle.levels(m)
    assert nl == len(g["wavefronts"]) == 4
    for w, members in enumerate(g["wavefronts"]):
        assert sorted(lab[i] for i in range(m.n) if lv[i] == w + 1) == sorted(members)
    # average wavefront size n / longest path, rounded down as in the tables
    assert oracle.avg_wavefront(m) == 1
    # vertex weights = stored entries per row (Sec. 2.2)
    assert np.diff(m.row_ptr).tolist() == [1, 2, 2, 2, 2, 2]


def test_fig_1_1_growlocal_single_superstep():
    """n <= alpha0 = 20: core 1 can take every vertex in the first iteration,
    which is saturated, so the schedule is one superstep on one core."""
    g = load_golden("fig1_1.json")
    m = gen.from_entries(g["n"], g["nonzeros_1based"])
    pi, sigma, S = oracle.growlocal(m, 22)
    assert S == 1 and not pi.any() and not sigma.any()
    perm, _ = oracle.reorder(m, pi, sigma)
    assert perm.tolist() == list(range(6))


def test_fig_3_1_blocks():
    g = load_golden("fig3_1.json")
    m = gen.from_entries(g["n"], g["nonzeros_1based"])
    assert oracle.check_csr(m) == 0
    # each diagonal block is itself lower triangular; its sub-DAG keeps the
    # edges between its own rows
    for lo, hi in g["diagonal_blocks_1based"]:
        for i in range(lo - 1, hi):
            for e in range(m.row_ptr[i], m.row_ptr[i + 1]):
                assert m.col[e] <= i
    pi, sigma, S = oracle.growlocal(m, 22)
    assert S == 1 and not pi.any()


# --------------------------------------------------------------------------
# closed forms derived by hand from the rules
# --------------------------------------------------------------------------

def test_edgeless_n1000_k4_L500():
    """Edgeless DAG, unit weights, k=4, L=500.  Superstep 1: alpha = 20, 30,
    45, 67.5, 101.25, 151.875, 227.8125 give cores [a, a, a, a] and
    beta = 4a / (a + 500); alpha = 341.71875 gives [341, 341, 318, 0],
    beta = 1000/841 < 0.97 * 908/727, so [227]*4 is kept.  Superstep 2 (92
    left): [20]*4 -> 80/520; [30,30,30,2] -> 92/530; [45,45,2,0] -> 92/545,
    worthy (>= 0.97 * 92/530) though lower; [67,25,0,0] -> 92/567 is not, so
    the last worthy one, [45,45,2,0], is kept."""
    m = gen.edgeless(1000)
    pi, sigma, S, tr = oracle.growlocal(m, 4, trace=64)
    assert S == 2
    assert counts_per_superstep(pi, sigma, S, 4) == [[227] * 4, [45, 45, 2, 0]]
    exp = [(0, 20.0, 80 / 520, True), (0, 30.0, 120 / 530, True), (0, 45.0, 180 / 545, True),
           (0, 67.5, 268 / 567, True), (0, 101.25, 404 / 601, True), (0, 151.875, 604 / 651, True),
           (0, 227.8125, 908 / 727, True), (0, 341.71875, 1000 / 841, False),
           (1, 20.0, 80 / 520, True), (1, 30.0, 92 / 530, True), (1, 45.0, 92 / 545, True),
           (1, 67.5, 92 / 567, False)]
    assert tr == exp
    # smallest IDs first, cores filled in order
    assert pi[:227].tolist() == [0] * 227 and pi[227:454].tolist() == [1] * 227


def test_edgeless_n100_k3_L0():
    m = gen.edgeless(100)
    pi, sigma, S = oracle.growlocal(m, 3, L=0.0)
    assert S == 2
    assert counts_per_superstep(pi, sigma, S, 3) == [[30, 30, 30], [10, 0, 0]]


def edgeless_model(n, k, L, alpha0, growth, theta):
    """The rules of Algorithm 3.1 on an edgeless DAG with unit weights, where
    every vertex is free at every barrier: core 1 takes min(floor(alpha),
    left) vertices, every later core the same count (its weight must reach
    core 1's), smallest IDs first."""
    left, out = n, []
    while left:
        alpha, best, kept, it = alpha0, 0.0, None, 0
        while True:
            a = min(math.floor(alpha), left)
            cnt, rest = [], left
            for _ in range(k):
                if not rest:
                    break
                c = min(a, rest)
                cnt.append(c)
                rest -= c
            beta = float(sum(cnt)) / (float(max(cnt)) + L)
            if it > 0 and not (beta >= theta * best):
                break
            kept = cnt
            if it == 0 or beta > best:
                best = beta
            if cnt[0] < math.floor(alpha):
                break
            alpha = growth * alpha
            it += 1
        out.append(kept + [0] * (k - len(kept)))
        left -= sum(kept)
    return out


@pytest.mark.parametrize("n,k,L,a0,g,th", [
    (1000, 4, 500.0, 20.0, 1.5, 0.97), (777, 5, 100.0, 3.0, 1.5, 0.97), (5000, 22, 500.0, 20.0, 1.5, 0.97),
    (300, 7, 0.0, 1.0, 2.0, 0.9), (12345, 64, 50.0, 1.0, 1.5, 0.97), (999, 1, 500.0, 20.0, 1.5, 0.97),
    (64, 100, 10.0, 2.0, 1.25, 0.99), (2048, 3, 1e4, 7.0, 1.7, 0.5)])
def test_edgeless_matches_independent_model(n, k, L, a0, g, th):
    m = gen.edgeless(n)
    pi, sigma, S = oracle.growlocal(m, k, L=L, alpha0=a0, growth=g, theta=th)
    assert counts_per_superstep(pi, sigma, S, k) == edgeless_model(n, k, L, a0, g, th)


@pytest.mark.parametrize("k,L", [(1, 500.0), (22, 500.0), (4, 0.0), (1000, 3.0)])
def test_chain_is_one_superstep(k, L):
    """A path DAG: every ready vertex is exclusive to core 1, beta grows with
    alpha (or stays 1 when L = 0), so core 1 saturates with the whole chain."""
    m = gen.chain(1000)
    pi, sigma, S = oracle.growlocal(m, k, L=L)
    assert S == 1 and not pi.any()


def test_rule_one_prefers_exclusive_vertices():
    """40 sources 0..39 plus vertex 40 with parents 0 and 1; k=2, L=0.
    alpha=20: core 1 takes 0, 1, then 40 (exclusive to it once 0 and 1 are
    placed) before the free 2..18; its weight is 19 + 3 = 22, so core 2 takes
    the 21 remaining sources 19..39: beta = 43/22.  alpha=30: core 1 takes 0,
    1, 40, 2..28 (weight 32), core 2 takes 29..39: beta = 43/32 < 0.97*43/22,
    so the alpha=20 superstep is kept and S = 1."""
    m = gen.from_entries(41, [(41, 1), (41, 2)])
    pi, sigma, S = oracle.growlocal(m, 2, L=0.0)
    assert S == 1
    assert pi[40] == 0 and (pi[:19] == 0).all() and (pi[19:40] == 1).all()


def test_rule_parents_on_two_cores_block():
    """40 sources plus vertex 40 with parents 0 and 39; k=2, L=0.  alpha=20:
    cores take 0..19 and 20..39, so vertex 40 has parents on two cores and
    must wait for the barrier; beta = 40/20.  alpha=30: [30, 10] -> 40/30 is
    not worthy, so S = 2 with vertex 40 alone in superstep 2."""
    m = gen.from_entries(41, [(41, 1), (41, 40)])
    pi, sigma, S = oracle.growlocal(m, 2, L=0.0)
    assert S == 2
    assert sigma[40] == 1 and (sigma[:40] == 0).all()
    assert (pi[:20] == 0).all() and (pi[20:40] == 1).all()


def test_single_source_grid_is_serial_under_the_literal_rules():
    """With one source, every vertex becomes exclusive to core 1, and beta =
    Omega/(Omega + L) only grows with alpha: the literal rules schedule a
    natural-order grid as one superstep on one core, for any L > 0."""
    m = gen.stencil_2d5(30)
    for L in (500.0, 50.0, 1.0):
        pi, sigma, S = oracle.growlocal(m, 22, L=L, alpha0=1.0)
        assert S == 1 and not pi.any()


# --------------------------------------------------------------------------
# invariants on random DAGs
# --------------------------------------------------------------------------

PARAMS = [dict(k=1), dict(k=2, L=0.0), dict(k=3, L=10.0, alpha0=1.0), dict(k=22),
          dict(k=100, L=50.0, alpha0=2.0), dict(k=4096, L=20.0, alpha0=1.0, growth=2.0, theta=0.9)]


def random_dags():
    out = []
    for s in range(10):
        out.append(gen.random_lower(120, 0.03 + 0.01 * s, 700 + s))
        out.append(gen.random_lower(200, 0.2, 800 + s, band=6))
    out += [gen.erdos_renyi(3000, 0.002, 901), gen.narrow_band(3000, 0.05, 20.0, 902), gen.stencil_2d5(20, 7)]
    return out


@pytest.mark.parametrize("pidx", range(len(PARAMS)))
def test_growlocal_schedules_are_valid(pidx):
    p = PARAMS[pidx]
    for m in random_dags():
        pi, sigma, S = oracle.growlocal(m, **p)
        assert oracle.validate(m, p["k"], pi, sigma, S) == oracle.VALID, m.name
        assert sorted(set(sigma.tolist())) == list(range(S))


def kahn_layers(m):
    """Wavefronts by repeatedly removing the sources (Kahn), independent of
    the oracle's longest-path recurrence."""
    indeg = np.diff(m.row_ptr) - 1
    kids = [[] for _ in range(m.n)]
    for i in range(m.n):
        for e in range(m.row_ptr[i], m.row_ptr[i + 1] - 1):
            kids[m.col[e]].append(i)
    layer = [i for i in range(m.n) if indeg[i] == 0]
    level = np.zeros(m.n, dtype=np.int64)
    d = 0
    while layer:
        d += 1
        nxt = []
        for v in layer:
            level[v] = d
            for u in kids[v]:
                indeg[u] -= 1
                if indeg[u] == 0:
                    nxt.append(u)
        layer = nxt
    return level, d


def test_levels_match_kahn_layering():
    for m in random_dags()[:12]:
        lv, nl = oracle.levels(m)
        lk, dk = kahn_layers(m)
        assert nl == dk and np.array_equal(lv, lk)


# --------------------------------------------------------------------------
# Definition 2.1 and strict-visibility execution
# --------------------------------------------------------------------------

def test_validator_and_bsp_catch_planted_errors():
    m = gen.erdos_renyi(2000, 0.004, 55)
    b = gen.rhs_uniform(m.n, 56)
    pi, sigma, S = oracle.growlocal(m, 8, L=20.0, alpha0=2.0)
    assert oracle.validate(m, 8, pi, sigma, S) == oracle.VALID
    x = oracle.bsp_solve(m, b, pi, sigma)
    assert oracle.same_bits(x, oracle.solve(m, b))
    # an edge (u, v) across cores: pull v into u's superstep
    for v in range(m.n):
        us = [int(m.col[e]) for e in range(m.row_ptr[v], m.row_ptr[v + 1] - 1) if pi[m.col[e]] != pi[v]]
        if us:
            u = us[0]
            break
    bad = sigma.copy()
    bad[v] = sigma[u]
    assert oracle.validate(m, 8, pi, bad, S) in (oracle.INVALID_CROSS, oracle.INVALID_ORDER)
    with pytest.raises(oracle.OracleError):
        oracle.bsp_solve(m, b, pi, bad)
    bad2 = sigma.copy()
    bad2[v] = sigma[u] - 1 if sigma[u] > 0 else 0
    if bad2[v] < sigma[u]:
        assert oracle.validate(m, 8, pi, bad2, S) == oracle.INVALID_ORDER
    bad3 = pi.copy()
    bad3[0] = 8
    assert oracle.validate(m, 8, bad3, sigma, S) == oracle.INVALID_RANGE


def test_wavefront_schedule_is_valid_and_exact():
    for m in random_dags()[:8]:
        pi, sigma, S = oracle.wavefront_schedule(m)
        assert oracle.validate(m, int(pi.max()) + 1, pi, sigma, S) == oracle.VALID
        b = gen.rhs_uniform(m.n, 3)
        assert oracle.same_bits(oracle.bsp_solve(m, b, pi, sigma), oracle.solve(m, b))


# --------------------------------------------------------------------------
# reordering (Sec. 5)
# --------------------------------------------------------------------------

def test_reorder_properties():
    for m in random_dags()[:10]:
        pi, sigma, S = oracle.growlocal(m, 5, L=10.0, alpha0=2.0)
        perm, (rp, col, val) = oracle.reorder(m, pi, sigma)
        assert sorted(perm.tolist()) == list(range(m.n))
        # order = sort by (superstep, core, original index)
        assert np.array_equal(perm, np.lexsort((np.arange(m.n), pi, sigma)))
        # still lower triangular, diagonal last, entries in their original order
        for t in range(m.n):
            cs = col[rp[t]:rp[t + 1]]
            assert cs[-1] == t and (cs[:-1] < t).all()
        pm = gen.CSR(m.n, rp, col, val)
        b = gen.rhs_uniform(m.n, 9)
        x = oracle.solve(m, b)
        # the permuted system gives the same values, row by row
        assert oracle.same_bits(oracle.solve(pm, b[perm]), x[perm])


# ---------------------------------------------------------------------------
# block-parallel scheduling, Sec. 3.1
# ---------------------------------------------------------------------------

def test_blocks_one_block_is_plain_growlocal():
    for m in (gen.random_lower(400, 0.02, 5), gen.fig_3_1(), gen.chain(50)):
        for k in (1, 3, 22):
            a = oracle.growlocal(m, k)
            b = oracle.growlocal_blocks(m, k, 1)
            assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _direct_sum(parts):
    """Block-diagonal matrix of the given lower-triangular pieces."""
    rp, cols, vals, off = [0], [], [], 0
    for m in parts:
        for i in range(m.n):
            for e in range(m.row_ptr[i], m.row_ptr[i + 1]):
                cols.append(int(m.col[e]) + off)
                vals.append(float(m.val[e]))
            rp.append(len(cols))
        off += m.n
    return gen.CSR(off, np.array(rp, np.int64), np.array(cols, np.int32), np.array(vals))


def test_blocks_of_a_direct_sum_are_the_pieces_scheduled_alone():
    # with no edge between blocks, each block is the piece itself (same DAG,
    # same weights), and the pieces' schedules follow one another
    pieces = [gen.random_lower(120, 0.05, 31), gen.random_lower(120, 0.02, 32), gen.chain(120)]
    m = _direct_sum(pieces)
    for k, L in ((2, 0.0), (4, 10.0), (22, 500.0)):
        pi, sg, S = oracle.growlocal_blocks(m, k, 3, L=L, alpha0=1.0)
        off = 0
        for b, piece in enumerate(pieces):
            p2, s2, S2 = oracle.growlocal(piece, k, L=L, alpha0=1.0)
            assert np.array_equal(pi[120 * b:120 * (b + 1)], p2)
            assert np.array_equal(sg[120 * b:120 * (b + 1)], s2 + off)
            off += S2
        assert S == off


def test_blocks_keep_the_weights_of_the_full_rows():
    # n = 6 in two blocks; row 3 stores entries in columns 0, 1, 2 (outside
    # its block) and 3, so its weight is 4 although its block DAG has no edge.
    # k = 2, L = 0, alpha0 = 1, growth 1.5, theta 0.97, derived by hand:
    # block 0 (rows 0-2, edgeless, weight 1): alpha 1 and 1.5 give
    #   {0 -> core 0, 1 -> core 1}, beta 2; alpha 2.25 gives beta 3/2 < 0.97*2,
    #   so superstep 0 = {0, 1}; superstep 1 = {2 -> core 0} (saturated).
    # block 1 (rows 3-5): alpha 1 and 1.5: core 0 takes 3 (weight 4), core 1
    #   takes 4 and 5 (weights 1, total 2 < 4), beta 6/4; alpha 2.25: core 0
    #   takes 3 and 4 (weight 5), core 1 takes 5, beta 6/5 < 0.97 * 1.5, so the
    #   whole block is superstep 2.  With the block's own row lengths (weight
    #   1 for row 3) row 5 would wait for a second superstep.
    m = gen.from_entries(6, [(4, 1), (4, 2), (4, 3)])   # 1-based (row, col)
    pi, sg, S = oracle.growlocal_blocks(m, 2, 2, L=0.0, alpha0=1.0)
    assert S == 3
    assert list(sg) == [0, 0, 1, 2, 2, 2]
    assert list(pi) == [0, 1, 0, 0, 1, 1]


@pytest.mark.parametrize("nblocks", [2, 3, 7, 50])
def test_block_schedules_are_valid_and_solve_exactly(nblocks):
    for s in range(4):
        m = gen.random_lower(300, 0.03, 60 + s, band=None if s % 2 else 12)
        for k, L, a0 in ((3, 0.0, 1.0), (22, 500.0, 20.0), (1 << 16, 50.0, 1.0)):
            pi, sg, S = oracle.growlocal_blocks(m, k, nblocks, L=L, alpha0=a0)
            assert oracle.validate(m, k, pi, sg, S) == oracle.VALID
            # every block's supersteps lie after those of the earlier blocks
            bounds = oracle.block_bounds(m.n, nblocks)
            for lo, mid, hi in zip(bounds[:-2], bounds[1:-1], bounds[2:]):
                if lo < mid < hi:
                    assert sg[lo:mid].max() < sg[mid:hi].min()
            b = gen.rhs_uniform(m.n, s)
            assert oracle.same_bits(oracle.bsp_solve(m, b, pi, sg), oracle.solve(m, b))
