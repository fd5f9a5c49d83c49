"""Seeded synthetic inputs for the sparse lower-triangular solve.

This module only *produces* inputs: sparsity patterns, matrix values and
right-hand sides.  It holds none of the solver's or the scheduler's
arithmetic, so both the CPU oracle (test infrastructure) and the HIP path
may draw their inputs from it.

Workload families (all return CSR with sorted columns, diagonal last):

* ``erdos_renyi``  -- Sec. 6.2.4 of the paper: every strictly-lower entry is
  non-zero independently with a fixed probability; off-diagonal values
  uniform in [-2, 2]; diagonal magnitude log-uniform in [1/2, 2] with a fair
  random sign.  The per-entry probability ``q`` is an argument; the paper's
  set (Table A.4 statistics) is reproduced with ``q = 2p`` (see
  ``erdos_renyi_paper``).
* ``narrow_band``  -- Sec. 6.2.5: entry (i, j), i > j, is non-zero with
  probability ``p * exp((1 + j - i) / B)``; same value distribution.
* ``stencil_*``    -- lower triangles of 2-D/3-D Laplacian stencils in natural
  order, stand-ins for the application matrices of Table A.1 (off-diagonal
  -1, diagonal 4 / 6 / 26).
* small fixed patterns: the 6x6 matrix of Fig. 1.1, the 9x9 matrix of
  Fig. 3.1, edgeless (diagonal) and chain (bidiagonal) matrices, and random
  small lower-triangular patterns for property tests.

Randomness comes from numpy's PCG64 generator seeded per instance; instance
``i`` of a family uses seed ``SEED_BASE + i``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2503054080


@dataclass
class CSR:
    """Square triangular matrix in CSR form.

    ``row_ptr`` int64[n+1], ``col`` int32[nnz], ``val`` float64[nnz].  Within a
    row the columns ascend; the diagonal entry is the last one of a lower
    triangle (the default) and the first one of an upper triangle
    (``meta["upper"]`` true, see :func:`upper_of`).
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def with_values(self, val: np.ndarray, name: str | None = None) -> "CSR":
        return CSR(self.n, self.row_ptr, self.col, np.ascontiguousarray(val, dtype=np.float64),
                   name if name is not None else self.name, dict(self.meta))


# ----------------------------------------------------------------------------
# assembly helpers
# ----------------------------------------------------------------------------

def _assemble(n: int, rows: np.ndarray, cols: np.ndarray, offvals: np.ndarray,
              diag: np.ndarray, name: str, presorted: bool = False) -> CSR:
    """Build CSR from strictly-lower (row, col, value) triples plus a diagonal.

    Triples may come in any order unless ``presorted``; duplicates are not
    allowed (callers generate distinct positions).
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    offvals = np.asarray(offvals, dtype=np.float64)
    if rows.size:
        assert (cols < rows).all() and (cols >= 0).all(), "strictly lower entries expected"
    if not presorted and rows.size:
        order = np.lexsort((cols, rows))
        rows, cols, offvals = rows[order], cols[order], offvals[order]
    counts = np.bincount(rows, minlength=n).astype(np.int64) + 1  # + diagonal
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    diag_pos = row_ptr[1:] - 1
    is_diag = np.zeros(nnz, dtype=bool)
    is_diag[diag_pos] = True
    col[~is_diag] = cols
    val[~is_diag] = offvals
    col[diag_pos] = np.arange(n, dtype=np.int32)
    val[diag_pos] = diag
    return CSR(n, row_ptr, col, val, name)


def paper_values(rng: np.random.Generator, m_off: int, n: int):
    """Value distribution of Sec. 6.2.4: off-diagonals U[-2, 2]; diagonal
    magnitude exp(U[ln 1/2, ln 2]) with a fair random sign."""
    off = rng.uniform(-2.0, 2.0, size=m_off)
    mag = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=n))
    sign = np.where(rng.integers(0, 2, size=n) == 1, 1.0, -1.0)
    return off, mag * sign


def _tri_index_to_rc(pos: np.ndarray):
    """Map a flat index over the strict lower triangle (row-major:
    pos = i(i-1)/2 + j, 0 <= j < i) back to (i, j): i is the last row whose
    first index i(i-1)/2 does not exceed pos (an exact integer search)."""
    pos = np.asarray(pos, dtype=np.int64)
    if pos.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    top = int(pos.max())
    imax = int(math.isqrt(2 * top)) + 2          # i(i-1)/2 > top for i = imax
    r = np.arange(imax + 1, dtype=np.int64)
    starts = r * (r - 1) // 2
    i = np.searchsorted(starts, pos, side="right").astype(np.int64) - 1
    j = pos - starts[i]
    assert ((j >= 0) & (j < i)).all()
    return i, j


def _bernoulli_positions(rng: np.random.Generator, total: int, prob: float, block: int = 1 << 22):
    """Sorted positions in [0, total) each chosen independently with
    probability ``prob`` (geometric skipping)."""
    if prob <= 0.0 or total <= 0:
        return np.zeros(0, dtype=np.int64)
    if prob >= 1.0:
        return np.arange(total, dtype=np.int64)
    out = []
    last = -1
    while True:
        expect = int((total - last) * prob)
        size = max(1024, min(block, int(expect * 1.05) + 64))
        gaps = rng.geometric(prob, size=size).astype(np.int64)
        pos = last + np.cumsum(gaps)
        keep = pos < total
        if not keep.all():
            out.append(pos[keep])
            break
        out.append(pos)
        last = int(pos[-1])
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


# ----------------------------------------------------------------------------
# random families of the paper
# ----------------------------------------------------------------------------

def erdos_renyi(n: int, q: float, seed: int, name: str | None = None) -> CSR:
    """Lower-triangular Erdos-Renyi matrix: each (i, j), i > j, non-zero with
    probability ``q`` (Sec. 6.2.4)."""
    rng = np.random.default_rng(seed)
    total = n * (n - 1) // 2
    pos = _bernoulli_positions(rng, total, q)
    rows, cols = _tri_index_to_rc(pos)
    off, diag = paper_values(rng, rows.size, n)
    m = _assemble(n, rows, cols, off, diag, name or f"ER_n{n}_q{q:g}_s{seed}", presorted=True)
    m.meta.update(family="ER", q=q, seed=seed)
    return m


def erdos_renyi_paper(n: int, p: float, seed: int) -> CSR:
    """The paper's ER set with the per-entry probability read as ``q = 2p``:
    this reproduces the off-diagonal counts and average wavefront sizes of
    Table A.4 (a literal ``q = p`` gives half the non-zeros)."""
    m = erdos_renyi(n, 2.0 * p, seed, name=f"ER_n{n}_p{p:g}_s{seed}")
    m.meta["p"] = p
    return m


def narrow_band(n: int, p: float, B: float, seed: int, name: str | None = None) -> CSR:
    """Narrow-bandwidth matrix of Sec. 6.2.5: (i, j), i > j, non-zero with
    probability p * exp((1 + j - i) / B)."""
    rng = np.random.default_rng(seed)
    rows_l, cols_l = [], []
    # distance d = i - j >= 1 has probability p * exp((1 - d) / B); stop once the
    # expected number of entries beyond d is below 1e-6.
    dmax = int(math.ceil(B * math.log(max(n * p * B * 1e6, 1.0)))) + 1
    dmax = min(dmax, n - 1)
    for d in range(1, dmax + 1):
        pd = p * math.exp((1.0 - d) / B)
        idx = _bernoulli_positions(rng, n - d, pd)
        if idx.size:
            i = idx + d
            rows_l.append(i)
            cols_l.append(i - d)
    rows = np.concatenate(rows_l) if rows_l else np.zeros(0, np.int64)
    cols = np.concatenate(cols_l) if cols_l else np.zeros(0, np.int64)
    if rows.size:
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        rows, cols = rows[order], cols[order]
    off, diag = paper_values(rng, rows.size, n)
    m = _assemble(n, rows, cols, off, diag, name or f"NB_n{n}_p{p:g}_B{B:g}_s{seed}", presorted=True)
    m.meta.update(family="NB", p=p, B=B, seed=seed)
    return m


NB_PAIRS = ((0.14, 10.0), (0.05, 20.0), (0.03, 42.0))   # Sec. 6.2.5
ER_PROBS = (1e-4, 5e-4, 2e-3)                            # Sec. 6.2.4


# ----------------------------------------------------------------------------
# stencil stand-ins (natural order, Laplacian values)
# ----------------------------------------------------------------------------

def _stencil(dims, offsets, diag_value: float, name: str) -> CSR:
    """Lower triangle of a Laplacian stencil.  ``offsets`` are (dx, dy, dz)
    triples that point to lower-numbered neighbours in natural order
    idx = x + nx*(y + ny*z).  Each row lists its neighbours by rising
    column, then the diagonal."""
    nx, ny, nz = dims
    n = nx * ny * nz
    strides = (1, nx, nx * ny)
    offs = sorted(offsets, key=lambda o: o[0] * strides[0] + o[1] * strides[1] + o[2] * strides[2])
    lin = np.array([dx * strides[0] + dy * strides[1] + dz * strides[2] for dx, dy, dz in offs] + [0],
                   dtype=np.int64)

    def valid(idx):
        # [rows, len(offs) + 1]: neighbour inside the grid (the diagonal always)
        x = idx % nx
        y = (idx // nx) % ny
        z = idx // (nx * ny)
        ok = np.ones((idx.size, len(offs) + 1), dtype=bool)
        for j, (dx, dy, dz) in enumerate(offs):
            if dx:
                ok[:, j] &= (x + dx >= 0) & (x + dx < nx)
            if dy:
                ok[:, j] &= (y + dy >= 0) & (y + dy < ny)
            if dz:
                ok[:, j] &= (z + dz >= 0) & (z + dz < nz)
        return ok

    chunk = 1 << 20
    counts = np.empty(n, dtype=np.int64)
    for r0 in range(0, n, chunk):
        idx = np.arange(r0, min(n, r0 + chunk), dtype=np.int64)
        counts[r0:r0 + idx.size] = valid(idx).sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    vals = np.full(len(offs) + 1, -1.0)
    vals[-1] = diag_value
    for r0 in range(0, n, chunk):
        idx = np.arange(r0, min(n, r0 + chunk), dtype=np.int64)
        ok = valid(idx)
        a, b = row_ptr[r0], row_ptr[r0 + idx.size]
        col[a:b] = (idx[:, None] + lin[None, :])[ok].astype(np.int32)
        val[a:b] = np.broadcast_to(vals, ok.shape)[ok]
    m = CSR(n, row_ptr, col, val, name)
    m.meta.update(family="stencil", dims=dims)
    return m


def stencil_2d5(nx: int, ny: int | None = None) -> CSR:
    ny = nx if ny is None else ny
    return _stencil((nx, ny, 1), [(-1, 0, 0), (0, -1, 0)], 4.0, f"st2d5_{nx}x{ny}")


def stencil_3d7(m: int) -> CSR:
    return _stencil((m, m, m), [(-1, 0, 0), (0, -1, 0), (0, 0, -1)], 6.0, f"st3d7_{m}")


def stencil_3d27(m: int) -> CSR:
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dz < 0 or (dz == 0 and (dy < 0 or (dy == 0 and dx < 0))):
                    offs.append((dx, dy, dz))
    assert len(offs) == 13
    return _stencil((m, m, m), offs, 26.0, f"st3d27_{m}")


# ----------------------------------------------------------------------------
# small fixed patterns
# ----------------------------------------------------------------------------

# Fig. 1.1(a): non-zeros (row, col), 1-based, rows a..f.
FIG_1_1_ENTRIES = ((1, 1), (2, 1), (2, 2), (3, 2), (3, 3), (4, 2), (4, 4),
                   (5, 3), (5, 5), (6, 4), (6, 6))
# Fig. 3.1(a): 9x9 matrix split into three 3x3 diagonal blocks.
FIG_3_1_ENTRIES = ((1, 1), (2, 1), (2, 2), (3, 2), (3, 3), (4, 2), (4, 4),
                   (5, 3), (5, 5), (6, 4), (6, 6), (7, 7), (8, 8), (9, 9),
                   (8, 1), (8, 3), (7, 2), (7, 3), (9, 2), (9, 7), (7, 6))


def from_entries(n: int, entries, offval=None, diag=None, name: str = "") -> CSR:
    """CSR from 1-based (row, col) pairs (diagonal pairs are ignored; every
    row gets a diagonal).  Values default to integers: off-diagonal -1,
    diagonal 1."""
    pairs = sorted({(int(r) - 1, int(c) - 1) for r, c in entries if r != c})
    rows = np.array([p[0] for p in pairs], dtype=np.int64)
    cols = np.array([p[1] for p in pairs], dtype=np.int64)
    if offval is None:
        offval = -np.ones(rows.size)
    if diag is None:
        diag = np.ones(n)
    return _assemble(n, rows, cols, np.asarray(offval, dtype=np.float64),
                     np.asarray(diag, dtype=np.float64), name, presorted=True)


def fig_1_1() -> CSR:
    return from_entries(6, FIG_1_1_ENTRIES, name="fig1_1")


def fig_3_1() -> CSR:
    return from_entries(9, FIG_3_1_ENTRIES, name="fig3_1")


def edgeless(n: int) -> CSR:
    """Diagonal matrix (a DAG with no edges), diagonal 1."""
    return _assemble(n, np.zeros(0), np.zeros(0), np.zeros(0), np.ones(n), f"edgeless_{n}")


def chain(n: int) -> CSR:
    """Bidiagonal matrix: row i depends on row i-1 (a path DAG)."""
    r = np.arange(1, n, dtype=np.int64)
    return _assemble(n, r, r - 1, -np.ones(n - 1), np.ones(n), f"chain_{n}", presorted=True)


def random_lower(n: int, density: float, seed: int, values: str = "paper",
                 band: int | None = None) -> CSR:
    """Small random lower-triangular pattern for property tests.

    ``values``: "paper" (Sec. 6.2.4 distribution), "int_unit" (off-diagonal
    integers in {-2..2}\\{0}, diagonal 1), "int_pow2" (off-diagonal integers,
    diagonal +-2^e, e in {-2..2}).
    ``band``: restrict entries to i - j <= band.
    """
    rng = np.random.default_rng(seed)
    ii, jj = np.tril_indices(n, -1)
    if band is not None:
        keep = (ii - jj) <= band
        ii, jj = ii[keep], jj[keep]
    mask = rng.random(ii.size) < density
    rows, cols = ii[mask].astype(np.int64), jj[mask].astype(np.int64)
    if values == "paper":
        off, diag = paper_values(rng, rows.size, n)
    elif values == "int_unit":
        off = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=rows.size)
        diag = np.ones(n)
    elif values == "int_pow2":
        off = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=rows.size)
        diag = np.ldexp(1.0, rng.integers(-2, 3, size=n)) * np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0)
    else:
        raise ValueError(values)
    return _assemble(n, rows, cols, off, diag, f"rand_n{n}_d{density:g}_s{seed}_{values}")


# ----------------------------------------------------------------------------
# right-hand sides
# ----------------------------------------------------------------------------

def rhs_ones(n: int) -> np.ndarray:
    """b = all ones, as in the paper's timing runs (Sec. 6.1)."""
    return np.ones(n, dtype=np.float64)


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def rhs_int(n: int, seed: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n).astype(np.float64)


# ----------------------------------------------------------------------------
# named workload sets
# ----------------------------------------------------------------------------

def small_set(n: int = 10_000):
    """Six n=1e4 systems shaped like the paper's synthetic sets: ER keeping the
    paper's average degree (p' = p * 1e5 / n, q = 2p') and NB with the three
    (p, B) pairs.  Seeds SEED_BASE + 0..5."""
    out = []
    for i, p in enumerate(ER_PROBS):
        pp = p * 1e5 / n
        m = erdos_renyi(n, 2.0 * pp, SEED_BASE + i, name=f"ER_n{n}_p{pp:g}")
        out.append(m)
    for i, (p, B) in enumerate(NB_PAIRS):
        out.append(narrow_band(n, p, B, SEED_BASE + 3 + i, name=f"NB_n{n}_p{p:g}_B{B:g}"))
    return out


def paper_synthetic_set(n: int = 100_000, instances=range(10)):
    """The paper's ER and NB sets at paper size (Tables A.4, A.5): instance
    letters A..J map to seeds SEED_BASE + 0..9 (ER) and + 10..19 (NB)."""
    out = []
    for p in ER_PROBS:
        for i in instances:
            out.append(erdos_renyi_paper(n, p, SEED_BASE + i))
    for p, B in NB_PAIRS:
        for i in instances:
            out.append(narrow_band(n, p, B, SEED_BASE + 10 + i))
    return out


def batch_mix(count: int = 64, seed: int = SEED_BASE + 100, lo_exp: float = 3.0, hi_exp: float = 6.0):
    """Batching workload: ``count`` independent systems with n = floor(10^U[lo,hi])
    drawn from {ER with average degree log-U[2, 50], NB (one of the three
    pairs), 2-D 5-point, 3-D 7-point}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = max(1, int(math.floor(10.0 ** rng.uniform(lo_exp, hi_exp))))
        kind = int(rng.integers(0, 4))
        s = seed + 1 + i
        if kind == 0:
            deg = math.exp(rng.uniform(math.log(2.0), math.log(50.0)))
            q = min(1.0, 2.0 * deg / max(n - 1, 1))
            out.append(erdos_renyi(n, q, s, name=f"mix{i}_ER_n{n}_d{deg:.1f}"))
        elif kind == 1:
            p, B = NB_PAIRS[int(rng.integers(0, 3))]
            out.append(narrow_band(n, p, B, s, name=f"mix{i}_NB_n{n}_p{p:g}_B{B:g}"))
        elif kind == 2:
            side = max(1, int(round(math.sqrt(n))))
            out.append(stencil_2d5(side, max(1, n // side)))
            out[-1].name = f"mix{i}_" + out[-1].name
        else:
            side = max(1, int(round(n ** (1.0 / 3.0))))
            m = _stencil((side, side, max(1, n // (side * side))),
                         [(-1, 0, 0), (0, -1, 0), (0, 0, -1)], 6.0, f"mix{i}_st3d7_{side}")
            out.append(m)
    return out


def er_n1e7() -> CSR:
    """The single-system benchmark matrix: Erdos-Renyi as Sec. 6.2.4 with
    n = 1e7 and 10 off-diagonals per row on average (q = 20 / (n - 1))."""
    n = 10_000_000
    return erdos_renyi(n, 20.0 / (n - 1), SEED_BASE + 200, name="ER_n1e7_d10")


def upper_of(m: CSR, name: str | None = None) -> CSR:
    """The transpose of a lower-triangular CSR: an upper-triangular CSR whose
    row j holds the entries of column j (rising columns, diagonal first), with
    the same values."""
    n = m.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(m.row_ptr))
    cols = m.col.astype(np.int64)
    order = np.lexsort((rows, cols))          # by column of m, then row of m
    t_rows, t_cols, t_vals = cols[order], rows[order], m.val[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(t_rows, minlength=n), out=row_ptr[1:])
    out = CSR(n, row_ptr, t_cols.astype(np.int32), np.ascontiguousarray(t_vals), name or (m.name + "_T"),
              dict(m.meta))
    out.meta["upper"] = True
    return out
