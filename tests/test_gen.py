"""The seeded inputs: statistics of the paper's synthetic sets (Tables A.4
and A.5 print off-diagonal counts and average wavefront sizes per instance),
closed-form sizes of the stencil stand-ins, and determinism."""
import numpy as np
import pytest

import oracle
from paper_2503_05408_amd import gen

# (min, max) over the ten instances of each set, Table A.4 / A.5
TABLE_A4 = {1e-4: ((999_915, 1_001_551), (1_639, 1_886)),
            5e-4: ((4_996_501, 5_006_107), (395, 414))}
TABLE_A5 = {(0.14, 10.0): ((146_328, 147_412), (61, 132)),
            (0.05, 20.0): ((102_021, 103_152), (892, 1_369)),
            (0.03, 42.0): ((127_019, 127_774), (29, 67))}


def within(v, lo, hi, rel):
    return lo * (1 - rel) <= v <= hi * (1 + rel)


@pytest.mark.parametrize("p", sorted(TABLE_A4))
def test_erdos_renyi_matches_table_a4(p):
    (clo, chi), (wlo, whi) = TABLE_A4[p]
    m = gen.erdos_renyi_paper(100_000, p, gen.SEED_BASE + 1)
    assert within(m.nnz - m.n, clo, chi, 0.005)
    assert within(oracle.avg_wavefront(m), wlo, whi, 0.10)


@pytest.mark.parametrize("pair", sorted(TABLE_A5))
def test_narrow_band_matches_table_a5(pair):
    (clo, chi), (wlo, whi) = TABLE_A5[pair]
    m = gen.narrow_band(100_000, pair[0], pair[1], gen.SEED_BASE + 12)
    assert within(m.nnz - m.n, clo, chi, 0.01)
    assert within(oracle.avg_wavefront(m), wlo, whi, 0.15)


def test_value_distribution():
    m = gen.erdos_renyi(20_000, 0.001, 5)
    diag = m.val[m.row_ptr[1:] - 1]
    off = np.delete(m.val, m.row_ptr[1:] - 1)
    assert off.min() >= -2 and off.max() <= 2 and abs(off.mean()) < 0.05
    mag = np.abs(diag)
    assert mag.min() >= 0.5 and mag.max() <= 2.0
    assert abs(np.log(mag).mean()) < 0.02          # log-uniform on [ln 1/2, ln 2]
    assert 0.45 < (diag > 0).mean() < 0.55          # fair sign


def test_stencil_sizes():
    m = gen.stencil_2d5(50, 40)
    assert m.n == 2000 and m.nnz == 2000 + 49 * 40 + 50 * 39
    m = gen.stencil_3d7(12)
    assert m.nnz == 12 ** 3 + 3 * 12 * 12 * 11
    m = gen.stencil_3d27(9)
    # 13 lower neighbours per interior point; count exactly by offsets
    c = 9 ** 3
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dz < 0 or (dz == 0 and (dy < 0 or (dy == 0 and dx < 0))):
                    c += (9 - abs(dx)) * (9 - abs(dy)) * (9 - abs(dz))
    assert m.nnz == c
    assert oracle.check_csr(m) == 0
    _, nl = oracle.levels(gen.stencil_3d7(10))
    assert nl == 3 * 10 - 2


def test_seeded_determinism():
    a = gen.narrow_band(5000, 0.05, 20.0, 42)
    b = gen.narrow_band(5000, 0.05, 20.0, 42)
    c = gen.narrow_band(5000, 0.05, 20.0, 43)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not np.array_equal(a.col, c.col[:a.col.size]) or a.nnz != c.nnz
    for m in gen.small_set(2000) + gen.batch_mix(6, lo_exp=2.0, hi_exp=3.5):
        assert oracle.check_csr(m) == 0, m.name
