"""Seeded synthetic inputs for the permuted-SpMV workloads.

This module is the only code shared by the CPU oracle and the GPU path. It
draws matrices and vectors; it holds none of the method's arithmetic (no
permutation, histogram, entropy or product). Every generator is a pure
function of its seed.

The paper measures on SuiteSparse matrices (OPF 3754, LP OSA 07, MULT DCOP
01/03; Section 6) that are not available here. The generators below stand in
for them with the structures the paper describes: a mostly block-diagonal
matrix whose x reads stay close together (Section 7, OPF 3754), and rows
of skewed length clustered near the diagonal (LP OSA 07's heavy clustered
rows). Dense rows or columns are excluded, as Section 1 requires.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "from_entries", "block_clustered", "skewed_clustered", "heavy_clustered",
    "clustered_n4096", "clustered_n2m", "skewed_n4m", "batch_member", "serving_member",
    "random_csr", "vector", "uniform_fill",
]


@dataclass
class CSR:
    """Canonical CSR: row_ptr[nrows+1] int32, col[nnz] int32 strictly
    increasing within a row, val[nnz] float64 (Section 2)."""
    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def from_entries(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray,
                 vals: np.ndarray) -> CSR:
    """Assemble canonical CSR from distinct (row, col) entries in any order."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.argsort(rows * ncols + cols, kind="stable")
    rows, cols, vals = rows[order], cols[order], np.asarray(vals, np.float64)[order]
    counts = np.bincount(rows, minlength=nrows)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return CSR(nrows, ncols, rp.astype(np.int32), cols.astype(np.int32), vals)


def _dedupe(rows: np.ndarray, cols: np.ndarray, ncols: int, redraw) -> np.ndarray:
    """Redraw entries until all (row, col) pairs are distinct. `redraw(idx)`
    returns fresh columns for the entries at positions idx."""
    cols = cols.copy()
    check = np.arange(len(rows))
    while len(check):
        key = rows[check] * ncols + cols[check]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup_pos = np.nonzero(ks[1:] == ks[:-1])[0] + 1
        if len(dup_pos) == 0:
            break
        idx = check[order[dup_pos]]
        cols[idx] = redraw(idx)
        # only rows that held a duplicate can hold one after the redraw
        bad_rows = np.unique(rows[idx])
        check = np.nonzero(np.isin(rows, bad_rows))[0]
    return cols


def block_clustered(n: int, nnz_per_row, block: int, p_in: float, seed: int,
                    ncols: int | None = None) -> CSR:
    """Square (or n x ncols) matrix where each entry of row i lands, with
    probability p_in, in the diagonal block [block*floor(i/block), +block)
    and otherwise uniformly among the columns outside that block.

    nnz_per_row is an int (every row that long) or an int array per row.
    The in-block count per row is Binomial(len, p_in), capped by the block
    width, so the in-block fraction is p_in in expectation. Values U[-1, 1].
    """
    ncols = n if ncols is None else ncols
    rng = np.random.default_rng(seed)
    lens = np.broadcast_to(np.asarray(nnz_per_row, dtype=np.int64), (n,)).copy()
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    b0 = (rows // block) * block
    bw = np.minimum(b0 + block, ncols) - b0          # width of the row's own block
    lens_in = np.minimum(rng.binomial(lens, p_in), np.minimum(block, ncols))
    # position of each entry inside its row decides in-block vs outside
    starts = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=starts[1:])
    pos = np.arange(len(rows), dtype=np.int64) - starts[rows]
    inside = pos < lens_in[rows]
    outside_w = ncols - bw                           # columns outside the block

    def draw(idx):
        r = rng.random(len(idx))
        c_in = b0[idx] + np.floor(r * bw[idx]).astype(np.int64)
        ow = np.maximum(outside_w[idx], 1)
        u = np.floor(r * ow).astype(np.int64)
        c_out = np.where(u < b0[idx], u, u + bw[idx])
        return np.where(inside[idx], c_in, c_out)

    cols = draw(np.arange(len(rows)))
    cols = _dedupe(rows, cols, ncols, draw)
    vals = rng.uniform(-1.0, 1.0, size=len(rows))
    return from_entries(n, ncols, rows, cols, vals)


def skewed_clustered(n: int, mu: float, sigma: float, cap: int, spread: float,
                     seed: int) -> CSR:
    """Row lengths clamp(rint(exp(mu + sigma z)), 1, cap); each column is
    rint(i + spread * z'), redrawn until inside [0, n) and distinct in the row.
    Values U[-1, 1]."""
    rng = np.random.default_rng(seed)
    lens = np.clip(np.rint(np.exp(mu + sigma * rng.standard_normal(n))), 1, cap).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)

    def draw(idx):
        out = np.rint(rows[idx] + spread * rng.standard_normal(len(idx))).astype(np.int64)
        bad = np.nonzero((out < 0) | (out >= n))[0]
        while len(bad):
            out[bad] = np.rint(rows[idx[bad]] + spread * rng.standard_normal(len(bad))).astype(np.int64)
            bad = bad[(out[bad] < 0) | (out[bad] >= n)]
        return out

    cols = draw(np.arange(len(rows)))
    cols = _dedupe(rows, cols, n, draw)
    vals = rng.uniform(-1.0, 1.0, size=len(rows))
    return from_entries(n, n, rows, cols, vals)


def heavy_clustered(n: int, base_len: int, heavy_frac: float, heavy_len: int, spread: float,
                    seed: int) -> CSR:
    """A stand-in for a matrix with a few very heavy rows that are clustered
    (the paper's LP OSA 07, Section 5): every row has base_len entries except
    one contiguous band of heavy_frac * n rows with heavy_len entries each;
    columns are rint(i + spread * z) around the diagonal, distinct in a row.
    No row is dense (heavy_len << n). Values U[-1, 1]."""
    rng = np.random.default_rng(seed)
    lens = np.full(n, base_len, dtype=np.int64)
    start = int(rng.integers(0, max(1, n - int(heavy_frac * n))))
    lens[start:start + int(heavy_frac * n)] = heavy_len
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)

    def draw(idx):
        out = np.rint(rows[idx] + spread * rng.standard_normal(len(idx))).astype(np.int64)
        bad = np.nonzero((out < 0) | (out >= n))[0]
        while len(bad):
            out[bad] = np.rint(rows[idx[bad]] + spread * rng.standard_normal(len(bad))).astype(np.int64)
            bad = bad[(out[bad] < 0) | (out[bad] >= n)]
        return out

    cols = _dedupe(rows, draw(np.arange(len(rows))), n, draw)
    vals = rng.uniform(-1.0, 1.0, size=len(rows))
    return from_entries(n, n, rows, cols, vals)


def vector(n: int, seed: int, k: int = 1) -> np.ndarray:
    """x (k == 1, shape [n]) or X (shape [n, k], row-major), FP64 U[-1, 1]."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, size=(n, k))
    return v[:, 0].copy() if k == 1 else v


# --- the five workloads ----------------------------------------------------

def clustered_n4096(seed: int = 1) -> CSR:
    """n = 4096, 16 nnz per row, 90% (in expectation) inside the row's own
    64-wide diagonal block, the rest uniform outside it."""
    return block_clustered(4096, 16, 64, 0.9, seed)


def clustered_n2m(seed: int = 1, n: int = 2_000_000) -> CSR:
    """n = 2,000,000, 10 nnz per row, 90% (in expectation) inside the
    4096-row diagonal block, the rest uniform outside it."""
    return block_clustered(n, 10, 4096, 0.9, seed)


def skewed_n4m(seed: int = 1, n: int = 4_000_000) -> CSR:
    """n = 4,000,000, row lengths lognormal(mu=2, sigma=1) capped at 256,
    columns Gaussian (sigma = 2000) around the row index."""
    return skewed_clustered(n, 2.0, 1.0, 256, 2000.0, seed)


BATCH_K = (1, 2, 4, 8, 16)


def batch_member(index: int, seed_base: int = 1000) -> tuple[CSR, int]:
    """Matrix `index` of the 64-matrix batch: rows log-uniform in
    [10k, 500k], 8-32 nnz per row, 90% inside 4096-row diagonal blocks.
    Returns the matrix and its right-hand-side count k."""
    seed = seed_base + index
    rng = np.random.default_rng([seed, 7])
    n = int(np.floor(np.exp(rng.uniform(np.log(1e4), np.log(5e5)))))
    lens = rng.integers(8, 33, size=n)
    k = BATCH_K[int(rng.integers(0, len(BATCH_K)))]
    return block_clustered(n, lens, 4096, 0.9, seed), k


def serving_member(index: int, seed_base: int = 1000) -> CSR:
    """Matrix `index` of the 32-matrix serving pool: rows log-uniform in
    [50k, 2M]; even indices take the block-clustered structure, odd ones the
    skewed clustered structure."""
    seed = seed_base + index
    rng = np.random.default_rng([seed, 11])
    n = int(np.floor(np.exp(rng.uniform(np.log(5e4), np.log(2e6)))))
    if index % 2 == 0:
        return block_clustered(n, 10, 4096, 0.9, seed)
    return skewed_clustered(n, 2.0, 1.0, 256, 2000.0, seed)


# --- small cases for tests --------------------------------------------------

def random_csr(nrows: int, ncols: int, density: float, seed: int,
               empty_rows: float = 0.0, max_row: int | None = None) -> CSR:
    """Uniformly random sparsity with optional forced-empty rows."""
    rng = np.random.default_rng(seed)
    lens = rng.binomial(ncols, density, size=nrows) if ncols > 0 else np.zeros(nrows, np.int64)
    if max_row is not None:
        lens = np.minimum(lens, max_row)
    if empty_rows > 0:
        lens[rng.random(nrows) < empty_rows] = 0
    rows, cols = [], []
    for i, L in enumerate(lens):
        if L:
            c = rng.choice(ncols, size=int(L), replace=False)
            rows.append(np.full(L, i))
            cols.append(c)
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = np.zeros(0, np.int64)
        cols = np.zeros(0, np.int64)
    vals = rng.uniform(-1.0, 1.0, size=len(rows))
    return from_entries(nrows, ncols, rows, cols, vals)


def uniform_fill(n: int = 4096, g: int = 64, per_block: int = 16) -> CSR:
    """A matrix whose g x g block grid holds exactly per_block entries in
    every block. The row with local index l inside its block-row places one
    entry in each block-column (l + stride*t) mod g, t < per_block, with
    stride = g / per_block, so every block receives one entry per t.
    Requires n divisible by g and per_block dividing g. Values are 1.0."""
    bs = n // g
    assert bs * g == n and bs * per_block % g == 0
    stride = g // per_block if per_block <= g else 1
    rows, cols = [], []
    for r in range(n):
        local = r % bs
        for t in range(per_block):
            bj = (local + stride * t) % g
            rows.append(r)
            cols.append(bj * bs + (local * 7 + t) % bs)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    return from_entries(n, n, rows, cols, np.ones(len(rows)))
