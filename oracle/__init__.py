"""CPU oracle for the GrowLocal-scheduled sparse lower-triangular solve.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product package.  It shares no
code with the HIP library.  The arithmetic lives in ``oracle.c`` (plain C,
compiled with ``-ffp-contract=off`` so every binary64 operation is rounded on
its own); this module only marshals numpy arrays.

Each function cites the passage of the paper (arxiv 2503.05408) it follows:

* :func:`solve`      -- forward substitution, Eq. (2.1).
* :func:`solve_upper` -- backward substitution, its mirror (Sec. 2.2);
  :func:`mirror_upper` and :func:`growlocal_upper` schedule it.
* :func:`levels`     -- wavefronts; average wavefront size = floor(n / #levels)
  (Sec. 6.2; the appendix tables round down).
* :func:`validate`   -- Definition 2.1.
* :func:`growlocal`  -- Algorithm 3.1 (Sec. 3, Eq. (3.1); acceptance factor
  0.97 from the proof of Theorem 3.1 in Appendix B).
* :func:`growlocal_blocks` -- block-parallel scheduling (Sec. 3.1).
* :func:`reorder`    -- Sec. 5.
* :func:`bsp_solve`  -- the schedule executed superstep by superstep with
  strict visibility (Sec. 2.3).
* :func:`bsp_solve_parallel` -- the same schedule on host threads with a
  barrier per superstep (``executor.c``; the kind of CPU executor the paper
  times, Sec. 6.1): the benchmark's second CPU baseline.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_EXE_SRC = os.path.join(_HERE, "executor.c")
_EXE_LIB = os.path.join(_HERE, "libexecutor.so")
_exe = None
_lock = threading.Lock()
_lib = None

# paper parameters of GrowLocal: L = 500 (Sec. 3, footnote), alpha starts at 20
# and grows by 1.5 (Sec. 3), acceptance factor 0.97 (Appendix B)
PAPER_L = 500.0
PAPER_ALPHA0 = 20.0
PAPER_GROWTH = 1.5
PAPER_THETA = 0.97

VALID = 0
INVALID_RANGE = 1
INVALID_ORDER = 2
INVALID_CROSS = 3
INVALID_EMPTY = 4


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` and ``executor.c`` into
    ``libexecutor.so`` (OpenMP) with gcc."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           _EXE_SRC, "-o", _EXE_LIB + ".tmp"]
    if force or not os.path.exists(_EXE_LIB) or os.path.getmtime(_EXE_LIB) < os.path.getmtime(_EXE_SRC):
        subprocess.run(cmd, check=True)
        os.replace(_EXE_LIB + ".tmp", _EXE_LIB)
    return _LIB


def _load_executor():
    global _exe
    with _lock:
        if _exe is None:
            if not os.path.exists(_EXE_LIB) or os.path.getmtime(_EXE_LIB) < os.path.getmtime(_EXE_SRC):
                build(force=True)
            lib = ctypes.CDLL(_EXE_LIB)
            P = ctypes.c_void_p
            lib.executor_bsp_omp.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32, P, P,
                                             ctypes.c_int32]
            lib.executor_bsp_omp.restype = ctypes.c_int
            _exe = lib
    return _exe


class Executor:
    """A schedule prepared for :func:`executor.c`'s parallel run: the order of
    Sec. 5 (superstep, then core, then row index), the task boundaries in it
    and the first task of each superstep."""

    def __init__(self, m, pi, sigma):
        self.rp, self.c, self.v = _csr(m)
        self.n = int(m.n)
        pi = np.asarray(pi, dtype=np.int64)
        sigma = np.asarray(sigma, dtype=np.int64)
        order = np.lexsort((np.arange(self.n), pi, sigma)).astype(np.int32)
        s_o, c_o = sigma[order], pi[order]
        new_task = np.r_[True, (s_o[1:] != s_o[:-1]) | (c_o[1:] != c_o[:-1])] if self.n else np.zeros(0, bool)
        starts = np.flatnonzero(new_task)
        self.order = order
        self.task_beg = np.r_[starts, self.n].astype(np.int64)
        S = int(sigma.max()) + 1 if self.n else 0
        task_s = s_o[starts]
        self.super_task = np.searchsorted(task_s, np.arange(S + 1), side="left").astype(np.int32)
        self.S = S

    def solve(self, b, threads: int = 0):
        """x for right-hand side b; returns (x, threads used)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n, dtype=np.float64)
        used = _load_executor().executor_bsp_omp(self.n, _p(self.rp), _p(self.c), _p(self.v), _p(self.order),
                                                 _p(self.task_beg), _p(self.super_task), self.S, _p(b), _p(x),
                                                 int(threads))
        return x, int(used)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            lib.oracle_check_csr.argtypes = [i64, P, P, P]
            lib.oracle_solve.argtypes = [i64, P, P, P, P, P]
            lib.oracle_solve_upper.argtypes = [i64, P, P, P, P, P]
            lib.oracle_levels.argtypes = [i64, P, P, P]
            lib.oracle_levels.restype = i64
            lib.oracle_validate.argtypes = [i64, P, P, i32, P, P, i32]
            lib.oracle_growlocal.argtypes = [i64, P, P, i32, dbl, dbl, dbl, dbl, P, P, P,
                                             i64, P, P, P, P, P]
            lib.oracle_growlocal_weighted.argtypes = [i64, P, P, P, i32, dbl, dbl, dbl, dbl, P, P, P,
                                                      i64, P, P, P, P, P]
            lib.oracle_reorder.argtypes = [i64, P, P, P, P, P, P, P, P, P]
            lib.oracle_bsp_solve.argtypes = [i64, P, P, P, P, P, P, P, P]
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(m):
    rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(m.col, dtype=np.int32)
    v = np.ascontiguousarray(m.val, dtype=np.float64)
    return rp, c, v


class OracleError(RuntimeError):
    pass


def check_csr(m) -> int:
    rp, c, v = _csr(m)
    return _load().oracle_check_csr(m.n, _p(rp), _p(c), _p(v))


def solve(m, b) -> np.ndarray:
    """Serial forward substitution, Eq. (2.1): running subtraction in stored
    column order, then one division by the diagonal."""
    rp, c, v = _csr(m)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(m.n, dtype=np.float64)
    rc = _load().oracle_solve(m.n, _p(rp), _p(c), _p(v), _p(b), _p(x))
    if rc:
        raise OracleError(f"oracle_solve: {rc}")
    return x


def solve_upper(m, b) -> np.ndarray:
    """Serial backward substitution of an upper-triangular CSR (diagonal
    first in each row): rows from the last to the first, running subtraction
    in stored column order, one division (the mirror of Eq. (2.1), Sec. 2.2)."""
    rp, c, v = _csr(m)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(m.n, dtype=np.float64)
    rc = _load().oracle_solve_upper(m.n, _p(rp), _p(c), _p(v), _p(b), _p(x))
    if rc:
        raise OracleError(f"oracle_solve_upper: {rc}")
    return x


def mirror_upper(m, keep_order: bool = False):
    """The lower-triangular matrix J A J of an upper-triangular A, with J the
    reversal (row/column i -> n-1-i).  Row n-1-i holds row i's entries.  With
    keep_order the entries stay in A's stored order (columns then fall and
    the diagonal moves to the end); otherwise columns rise (a sorted CSR).
    Its DAG is A's DAG with every vertex renamed i -> n-1-i."""
    from paper_2503_05408_amd.gen import CSR
    rp, c, v = _csr(m)
    n = m.n
    rows_rp = np.zeros(n + 1, dtype=np.int64)
    lens = (rp[1:] - rp[:-1])[::-1]
    np.cumsum(lens, out=rows_rp[1:])
    col2 = np.empty_like(c)
    val2 = np.empty_like(v)
    for t in range(n):
        i = n - 1 - t
        a, e = rp[i], rp[i + 1]
        offc = (n - 1 - c[a + 1:e]).astype(np.int32)
        offv = v[a + 1:e]
        if not keep_order:
            offc, offv = offc[::-1], offv[::-1]
        o = rows_rp[t]
        col2[o:o + e - a - 1] = offc
        val2[o:o + e - a - 1] = offv
        col2[o + e - a - 1] = t
        val2[o + e - a - 1] = v[a]
    return CSR(n, rows_rp, col2, val2, name=(m.name or "") + "_mirror")


def growlocal_upper(m, k, L=PAPER_L, alpha0=PAPER_ALPHA0, growth=PAPER_GROWTH, theta=PAPER_THETA,
                    nblocks: int = 1):
    """GrowLocal for backward substitution: the DAG of an upper-triangular A
    with its vertices numbered in the direction of the solve (row i is
    vertex n-1-i), so Algorithm 3.1's smallest-ID rules and the diagonal
    blocks of Sec. 3.1 run in the reverse direction as the text prescribes.
    Returns (pi, sigma, S) indexed by the rows of A."""
    low = mirror_upper(m)
    if nblocks > 1:
        pi, sg, S = growlocal_blocks(low, k, nblocks, L=L, alpha0=alpha0, growth=growth, theta=theta)
    else:
        pi, sg, S = growlocal(low, k, L=L, alpha0=alpha0, growth=growth, theta=theta)
    return pi[::-1].copy(), sg[::-1].copy(), S


def levels(m):
    """(level per row, number of wavefronts); sources have level 1."""
    rp, c, _ = _csr(m)
    lv = np.empty(m.n, dtype=np.int32)
    nl = _load().oracle_levels(m.n, _p(rp), _p(c), _p(lv))
    if nl < 0:
        raise OracleError(f"oracle_levels: {nl}")
    return lv, int(nl)


def avg_wavefront(m) -> int:
    _, nl = levels(m)
    return m.n // nl if nl else 0


def validate(m, k, pi, sigma, S=None) -> int:
    rp, c, _ = _csr(m)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.int32)
    if S is None:
        S = int(sigma.max()) + 1 if m.n else 0
    return _load().oracle_validate(m.n, _p(rp), _p(c), int(k), _p(pi), _p(sigma), int(S))


def growlocal(m, k, L=PAPER_L, alpha0=PAPER_ALPHA0, growth=PAPER_GROWTH, theta=PAPER_THETA,
              trace: int = 0):
    """GrowLocal (Algorithm 3.1).  Returns (pi, sigma, S) and, when ``trace`` > 0,
    also a list of (superstep, alpha, beta, worthy) for the first ``trace``
    iterations."""
    rp, c, _ = _csr(m)
    pi = np.empty(m.n, dtype=np.int32)
    sigma = np.empty(m.n, dtype=np.int32)
    S = ctypes.c_int32(0)
    nt = ctypes.c_int64(0)
    if trace:
        ts = np.zeros(trace, np.int32)
        ta = np.zeros(trace, np.float64)
        tb = np.zeros(trace, np.float64)
        tw = np.zeros(trace, np.int8)
    else:
        ts = ta = tb = tw = None
    rc = _load().oracle_growlocal(m.n, _p(rp), _p(c), int(k), float(L), float(alpha0), float(growth),
                                  float(theta), _p(pi), _p(sigma), ctypes.byref(S), int(trace),
                                  _p(ts), _p(ta), _p(tb), _p(tw), ctypes.byref(nt))
    if rc:
        raise OracleError(f"oracle_growlocal: {rc}")
    if trace:
        cnt = min(trace, nt.value)
        tr = [(int(ts[i]), float(ta[i]), float(tb[i]), bool(tw[i])) for i in range(cnt)]
        return pi, sigma, S.value, tr
    return pi, sigma, S.value


def block_bounds(n: int, nblocks: int) -> list[int]:
    """Row bounds of the diagonal blocks: block b holds rows
    [floor(b n / B), floor((b+1) n / B)) (equal row counts; the paper does not
    say how the blocks are sized)."""
    return [(b * n) // nblocks for b in range(nblocks + 1)]


def growlocal_blocks(m, k, nblocks, L=PAPER_L, alpha0=PAPER_ALPHA0, growth=PAPER_GROWTH,
                     theta=PAPER_THETA):
    """Block-parallel GrowLocal (Sec. 3.1): the matrix is cut along the
    diagonal into ``nblocks`` lower-triangular blocks; each block is scheduled
    by Algorithm 3.1 as a DAG of its own (the edges from earlier blocks are
    dropped: those parents all finish in earlier supersteps) with the vertex
    weights of the full rows; the schedules are placed one after the other by
    adding to each block's superstep numbers the supersteps of all earlier
    blocks.  Returns (pi, sigma, S)."""
    rp, c, _ = _csr(m)
    pi = np.empty(m.n, dtype=np.int32)
    sigma = np.empty(m.n, dtype=np.int32)
    offset = 0
    bounds = block_bounds(m.n, nblocks)
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        if hi == lo:
            continue
        nb = hi - lo
        lens = rp[lo + 1:hi + 1] - rp[lo:hi]
        seg = np.repeat(np.arange(nb), lens)
        cols = c[rp[lo]:rp[hi]]
        keep = cols >= lo
        sub_rp = np.zeros(nb + 1, dtype=np.int64)
        np.cumsum(np.bincount(seg[keep], minlength=nb), out=sub_rp[1:])
        sub_col = np.ascontiguousarray(cols[keep] - lo, dtype=np.int32)
        weight = np.ascontiguousarray(lens, dtype=np.int64)
        pb = np.empty(nb, dtype=np.int32)
        sb = np.empty(nb, dtype=np.int32)
        S = ctypes.c_int32(0)
        nt = ctypes.c_int64(0)
        rc = _load().oracle_growlocal_weighted(nb, _p(sub_rp), _p(sub_col), _p(weight), int(k), float(L),
                                               float(alpha0), float(growth), float(theta), _p(pb), _p(sb),
                                               ctypes.byref(S), 0, None, None, None, None, ctypes.byref(nt))
        if rc:
            raise OracleError(f"oracle_growlocal_weighted: {rc}")
        pi[lo:hi] = pb
        sigma[lo:hi] = sb + offset
        offset += S.value
    return pi, sigma, offset


def wavefront_schedule(m):
    """The level-set schedule: superstep = level - 1, core = rank of the row
    inside its level (one row per core)."""
    lv, nl = levels(m)
    sigma = (lv - 1).astype(np.int32)
    order = np.argsort(sigma, kind="stable")           # by level, then ID
    start = np.zeros(nl + 1, dtype=np.int64)
    np.cumsum(np.bincount(sigma, minlength=nl), out=start[1:])
    pi = np.empty(m.n, dtype=np.int32)
    pi[order] = (np.arange(m.n) - start[sigma[order]]).astype(np.int32)
    return pi, sigma, nl


def reorder(m, pi, sigma):
    """Sec. 5: returns (perm, permuted CSR as (row_ptr, col, val)); row t of the
    permuted matrix is row perm[t] of A with columns renamed through the
    inverse permutation and the stored entry order kept."""
    rp, c, v = _csr(m)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.int32)
    perm = np.empty(m.n, dtype=np.int32)
    rp2 = np.empty(m.n + 1, dtype=np.int64)
    c2 = np.empty(m.nnz, dtype=np.int32)
    v2 = np.empty(m.nnz, dtype=np.float64)
    rc = _load().oracle_reorder(m.n, _p(rp), _p(c), _p(v), _p(pi), _p(sigma), _p(perm),
                                _p(rp2), _p(c2), _p(v2))
    if rc:
        raise OracleError(f"oracle_reorder: {rc}")
    return perm, (rp2, c2, v2)


def bsp_solve(m, b, pi, sigma):
    """Executes the schedule with strict visibility.  Returns x, or raises with
    the first row that read a value it could not yet see."""
    rp, c, v = _csr(m)
    b = np.ascontiguousarray(b, dtype=np.float64)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.int32)
    x = np.empty(m.n, dtype=np.float64)
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_bsp_solve(m.n, _p(rp), _p(c), _p(v), _p(b), _p(pi), _p(sigma), _p(x),
                                  ctypes.byref(bad))
    if rc:
        raise OracleError(f"oracle_bsp_solve: {rc} at row {bad.value}")
    return x


def bsp_solve_parallel(m, b, pi, sigma, threads: int = 0):
    """The schedule (pi, sigma) of a lower-triangular m executed on `threads`
    host threads (0 = the OpenMP default), superstep by superstep with a
    barrier between them, each task's rows in the order of Sec. 5 (see
    ``executor.c``).  The schedule must satisfy Definition 2.1 (check it with
    :func:`validate`).  Returns (x, threads used)."""
    return Executor(m, pi, sigma).solve(b, threads)


def same_bits(a, b) -> bool:
    """Comparison rule for binary64 results: bitwise equality (sign of zero
    included); two NaNs count as equal whatever their payload or sign."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    ia, ib = a.view(np.uint64), b.view(np.uint64)
    return bool(np.array_equal(ia[~na], ib[~nb]))


# ---------------------------------------------------------------------------
# Funnel coarsening (Sec. 4)
# ---------------------------------------------------------------------------

def _parents_children(m):
    """Parent and child lists of the DAG of a lower-triangular CSR (edge
    (j, i) for every stored off-diagonal A_ij)."""
    rp, c, _ = _csr(m)
    parents = [sorted({int(j) for j in c[rp[i]:rp[i + 1] - 1]}) for i in range(m.n)]
    children = [[] for _ in range(m.n)]
    for i in range(m.n):
        for j in parents[i]:
            children[j].append(i)
    return parents, children


def transitive_reduction(m):
    """Approximate transitive reduction of Sec. 4.2 ("remove all long edges
    in triangles"): an edge (u, w) is removed when some v has edges (u, v)
    and (v, w) in the original DAG.  Returns the kept parent lists."""
    parents, children = _parents_children(m)
    kept = []
    for w in range(m.n):
        pw = set(parents[w])
        kept.append([u for u in parents[w] if not any(v in pw for v in children[u])])
    return kept


def funnel_partition(m, max_weight):
    """In-funnel coarsening, Algorithm 4.1, on the transitively reduced DAG.
    Vertices are visited in reverse topological order (n-1 down to 0); the
    priority queue pops the largest vertex ID first; a parent joins once all
    of its children are in the part; a popped vertex that would lift the
    part's weight (stored entries of the rows) above max_weight is left out
    (it starts or joins a later part).  Returns part[v], parts numbered by
    their root (the vertex the part grew from) in rising order."""
    import heapq
    rp, _, _ = _csr(m)
    w_of = [int(rp[i + 1] - rp[i]) for i in range(m.n)]
    par = transitive_reduction(m)
    outdeg = [0] * m.n
    for w in range(m.n):
        for u in par[w]:
            outdeg[u] += 1
    visited = [False] * m.n
    part_root = {}
    roots = []
    for v in range(m.n - 1, -1, -1):
        if visited[v]:
            continue
        members, weight = [], 0
        count = {}
        heap = [-v]
        while heap:
            x = -heapq.heappop(heap)
            if weight + w_of[x] > max_weight and members:
                continue
            members.append(x)
            weight += w_of[x]
            for u in par[x]:
                count[u] = count.get(u, 0) + 1
                if count[u] == outdeg[u]:
                    heapq.heappush(heap, -u)
        for x in members:
            visited[x] = True
            part_root[x] = v
        roots.append(v)
    order = {r: i for i, r in enumerate(sorted(roots))}
    return np.array([order[part_root[v]] for v in range(m.n)], dtype=np.int32)


def coarse_dag(m, part):
    """Coarsened graph (Definition 4.1) of the transitively reduced DAG along
    the partition, as a lower-triangular pattern CSR over the parts (parts are
    numbered in a topological order: by root) with part weights = summed row
    weights.  Returns (CSR, weights)."""
    from paper_2503_05408_amd.gen import CSR
    rp, _, _ = _csr(m)
    par = transitive_reduction(m)
    P = int(part.max()) + 1 if m.n else 0
    cparents = [set() for _ in range(P)]
    weight = np.zeros(P, dtype=np.int64)
    for w in range(m.n):
        weight[part[w]] += rp[w + 1] - rp[w]
        for u in par[w]:
            if part[u] != part[w]:
                cparents[part[w]].add(int(part[u]))
    row_ptr = [0]
    col = []
    for q in range(P):
        ps = sorted(cparents[q])
        assert all(p < q for p in ps), "parts are not in topological order"
        col += ps + [q]
        row_ptr.append(len(col))
    return CSR(P, np.array(row_ptr, np.int64), np.array(col, np.int32), np.ones(len(col))), weight


def funnel_growlocal(m, k, max_weight, L=PAPER_L, alpha0=PAPER_ALPHA0, growth=PAPER_GROWTH, theta=PAPER_THETA):
    """Funnel + GrowLocal: Algorithm 3.1 on the coarsened DAG (part weights),
    pulled back so that every row takes its part's core and superstep.
    Returns (pi, sigma, S, part)."""
    part = funnel_partition(m, max_weight)
    cm, weight = coarse_dag(m, part)
    rp, c, _ = _csr(cm)
    P = cm.n
    pc = np.empty(P, dtype=np.int32)
    sc = np.empty(P, dtype=np.int32)
    S = ctypes.c_int32(0)
    nt = ctypes.c_int64(0)
    w = np.ascontiguousarray(weight, dtype=np.int64)
    rc = _load().oracle_growlocal_weighted(P, _p(rp), _p(c), _p(w), int(k), float(L), float(alpha0), float(growth),
                                           float(theta), _p(pc), _p(sc), ctypes.byref(S), 0, None, None, None,
                                           None, ctypes.byref(nt))
    if rc:
        raise OracleError(f"oracle_growlocal_weighted: {rc}")
    return pc[part].astype(np.int32), sc[part].astype(np.int32), S.value, part
