"""The seeded generators produce the workload structures they promise."""
import numpy as np

import synth


def _canonical(A):
    rp = A.row_ptr.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(A.col) == len(A.val)
    assert A.col.min(initial=0) >= 0 and A.col.max(initial=-1) < A.ncols
    rows = np.repeat(np.arange(A.nrows), np.diff(rp))
    same = rows[1:] == rows[:-1]
    assert np.all(np.diff(A.col.astype(np.int64))[same] > 0)


def test_clustered_n4096_structure():
    A = synth.clustered_n4096(1)
    _canonical(A)
    assert A.nrows == A.ncols == 4096 and np.all(A.row_lengths() == 16)
    rows = np.repeat(np.arange(4096), 16)
    frac = np.mean(A.col // 64 == rows // 64)
    assert abs(frac - 0.9) < 0.005          # Binomial(16, 0.9) per row
    assert np.all(np.abs(A.val) <= 1)
    B = synth.clustered_n4096(1)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_clustered_n2m_structure_small():
    A = synth.clustered_n2m(1, n=100_000)
    _canonical(A)
    assert np.all(A.row_lengths() == 10)
    rows = np.repeat(np.arange(A.nrows), 10)
    frac = np.mean(A.col // 4096 == rows // 4096)
    assert abs(frac - 0.9) < 0.003


def test_skewed_n4m_structure_small():
    A = synth.skewed_n4m(1, n=200_000)
    _canonical(A)
    L = A.row_lengths()
    assert L.min() >= 1 and L.max() <= 256
    assert abs(L.mean() - 12.18) < 0.25     # E[clamp(rint(e^(2+z)), 1, 256)]
    rows = np.repeat(np.arange(A.nrows), L)
    d = A.col.astype(np.int64) - rows
    inner = (rows > 10_000) & (rows < A.nrows - 10_000)
    assert abs(np.std(d[inner]) - 2000) < 40


def test_batch_and_serving_small_members():
    A, k = synth.batch_member(0)
    _canonical(A)
    assert 10_000 <= A.nrows <= 500_000 and k in synth.BATCH_K
    L = A.row_lengths()
    assert L.min() >= 8 and L.max() <= 32


def test_uniform_fill_is_uniform():
    U = synth.uniform_fill(4096, 64, 16)
    _canonical(U)
    rows = np.repeat(np.arange(4096), U.row_lengths())
    h = np.zeros((64, 64), int)
    np.add.at(h, (rows // 64, U.col // 64), 1)
    assert np.all(h == 16)


def test_heavy_clustered_structure():
    A = synth.heavy_clustered(20_000, 8, 0.02, 256, 2000.0, 3)
    _canonical(A)
    L = A.row_lengths()
    heavy = np.nonzero(L == 256)[0]
    assert len(heavy) == 400 and np.all(np.diff(heavy) == 1)      # one contiguous band
    assert np.all(L[L != 256] == 8)
