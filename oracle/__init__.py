"""CPU oracle for max-entropy permuted SpMV — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of every step the
GPU path computes, written from the paper (Jain et al., "Entropy
Maximization in Sparse Matrix by Vector Multiplication"). Only `tests/`,
`__graft_entry__.smoke()` and the benchmark's CPU-baseline leg may import it;
the product library never does, and the two share no code. The integer and
FP64 steps live in plain C (`mxe_oracle.c`, loaded with ctypes); the entropy
is evaluated here in 60-digit decimal arithmetic.

Parity status per function (what pins it is in tests/test_oracle.py):
  splitmix64_outputs, stream_seeds  pinned (published known answers)
  permutation, inverse              pinned (bijection, library argsort, chi-square)
  permute_csr, permute              pinned (scipy slicing, dense brute force)
  block_hist                        pinned (dense brute force, remap invariance)
  entropy                           pinned (closed forms, uniform fill, scipy)
  spmm / spmv                       pinned (dense brute force, scipy)
  coo_rows, coo_spmm                pinned (dense brute force, scipy COO, shuffled entry order)
  spmm_semiring                     pinned (dense brute force, scipy shortest paths, BFS reachability)
  entropy_levels                    pinned (uniform fill per level, hand cases, L = 1 is the global H)
  gradient_permutation, permute_gradient
                                    pinned (hand-built step profile, ties, edges, scipy slicing)
  round_f32, round_bf16             pinned (IEEE halfway cases, torch for FP32-exact inputs)
  bf16_to_f64                       pinned (hand-decoded bit patterns, torch on all 65536)
  stored_values                     pinned (numpy float32 rounding, golden BF16 cases decoded
                                    by Python's binary32 unpacking, torch on FP32-exact inputs)
  normalized_error                  pinned (hand cases)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from decimal import Decimal, localcontext

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mxe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ROWS = 1
COLS = 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _c():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.orc_splitmix64_outputs.argtypes = [u64, i64, P]
        lib.orc_stream_seeds.argtypes = [u64, P, P]
        lib.orc_argsort_keys.argtypes = [i64, P, P]
        lib.orc_argsort_keys.restype = ctypes.c_int
        lib.orc_invert.argtypes = [i64, P, P]
        lib.orc_permute_csr.argtypes = [i32, P, P, P, P, P, P, P, P]
        lib.orc_permute_csr.restype = ctypes.c_int
        lib.orc_block_hist.argtypes = [i32, i32, P, P, i32, i32, P]
        lib.orc_spmm.argtypes = [i32, P, P, P, i32, P, i64, P, i64]
        lib.orc_spmm_parallel.argtypes = [i32, P, P, P, i32, P, i64, P, i64]
        lib.orc_coo_spmm.argtypes = [i32, i64, P, P, P, i32, P, i64, P, i64]
        lib.orc_spmm_min_plus.argtypes = [i32, P, P, P, i32, P, i64, P, i64]
        lib.orc_spmm_or_and.argtypes = [i32, P, P, P, i32, P, i64, P, i64]
        lib.orc_omp_max_threads.restype = ctypes.c_int
        lib.orc_round_f32.argtypes = [i64, P, P]
        lib.orc_round_bf16.argtypes = [i64, P, P]
        lib.orc_bf16_from_f64.argtypes = [ctypes.c_double]
        lib.orc_bf16_from_f64.restype = ctypes.c_uint16
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c_i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _c_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- keys and permutations (Section 3, Eq. 1) -------------------------------

def splitmix64_outputs(state: int, n: int) -> np.ndarray:
    """First n outputs of SplitMix64 started at `state`."""
    out = np.empty(max(n, 0), dtype=np.uint64)
    _c().orc_splitmix64_outputs(ctypes.c_uint64(state & (2**64 - 1)), n, _p(out))
    return out


def stream_seeds(seed: int) -> tuple[int, int]:
    """(row stream seed, column stream seed) derived from the user seed."""
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _c().orc_stream_seeds(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def permutation(n: int, stream_seed: int) -> np.ndarray:
    """New-to-old random permutation of n items: stable argsort of the
    stream's first n SplitMix64 outputs."""
    keys = splitmix64_outputs(stream_seed, n)
    perm = np.empty(n, dtype=np.int32)
    if _c().orc_argsort_keys(n, _p(keys), _p(perm)) != 0:
        raise MemoryError("oracle argsort")
    return perm


def inverse(perm: np.ndarray) -> np.ndarray:
    perm = _c_i32(perm)
    inv = np.empty_like(perm)
    _c().orc_invert(len(perm), _p(perm), _p(inv))
    return inv


def permute_csr(A, rperm: np.ndarray, cperm: np.ndarray):
    """B = P_r A P_c in canonical CSR. Returns (row_ptr, col, val)."""
    rp, col, val = _c_i32(A.row_ptr), _c_i32(A.col), _c_f64(A.val)
    rperm = _c_i32(rperm)
    cinv = inverse(cperm)
    rp_o = np.empty(A.nrows + 1, np.int32)
    col_o = np.empty(len(col), np.int32)
    val_o = np.empty(len(val), np.float64)
    if _c().orc_permute_csr(A.nrows, _p(rp), _p(col), _p(val), _p(rperm), _p(cinv),
                            _p(rp_o), _p(col_o), _p(val_o)) != 0:
        raise MemoryError("oracle permute")
    return rp_o, col_o, val_o


def permute(A, seed: int, mode: int = ROWS | COLS):
    """The randomization of Section 3 for a user seed: rows permuted by the
    row stream when mode has ROWS, columns by the column stream when mode
    has COLS (identity otherwise). Returns (rperm, cperm, (rp, col, val))."""
    s_r, s_c = stream_seeds(seed)
    rperm = permutation(A.nrows, s_r) if mode & ROWS else np.arange(A.nrows, dtype=np.int32)
    cperm = permutation(A.ncols, s_c) if mode & COLS else np.arange(A.ncols, dtype=np.int32)
    return rperm, cperm, permute_csr(A, rperm, cperm)


# --- histogram and entropy (Sections 4 and 5) -------------------------------

def block_hist(nrows: int, ncols: int, row_ptr, col, grid_r: int, grid_c: int) -> np.ndarray:
    """G_r x G_c counts of stored entries (int64, shape [grid_r, grid_c])."""
    h = np.empty((grid_r, grid_c), dtype=np.int64)
    rp, c = _c_i32(row_ptr), _c_i32(col)
    _c().orc_block_hist(nrows, ncols, _p(rp), _p(c), grid_r, grid_c, _p(h))
    return h


def entropy(hist) -> tuple[float, float]:
    """Shannon entropy of the distribution p_i = h_i / S (Section 4, Eq.
    eq:entropy), bins with h_i = 0 contributing nothing. Evaluated in 60
    significant decimal digits and rounded once to the nearest double.
    Returns (bits, nats). An all-zero histogram has no distribution; the
    reading taken is H = 0."""
    h = np.asarray(hist, dtype=np.int64).ravel()
    S = int(h.sum())
    if S == 0:
        return 0.0, 0.0
    with localcontext() as ctx:
        ctx.prec = 60
        Sd = Decimal(S)
        lnp = {}
        total = Decimal(0)
        for hv in h[h > 0].tolist():
            p = Decimal(hv) / Sd
            if hv not in lnp:
                lnp[hv] = p.ln()
            total += p * lnp[hv]
        nats = -total
        bits = nats / Decimal(2).ln()
    return float(bits), float(nats)


def entropy_levels(hist, levels=(2, 4, 8)):
    """Hierarchical 2D entropy (Section 5): for each level L the G_r x G_c
    histogram is cut into min(L, G_r) x min(L, G_c) regions, region (a, b)
    holding the bins (r, c) with floor(r * Lr / G_r) = a and
    floor(c * Lc / G_c) = b, and each region's entropy is that of its own
    bins (Eq. 2). Returns a list of (bits, nats) arrays of shape [Lr, Lc]."""
    h = np.asarray(hist, dtype=np.int64)
    gr, gc = h.shape
    out = []
    for L in levels:
        lr, lc = min(L, gr), min(L, gc)
        bits = np.zeros((lr, lc))
        nats = np.zeros((lr, lc))
        for a in range(lr):
            rows = [r for r in range(gr) if r * lr // gr == a]
            for b in range(lc):
                cols = [c for c in range(gc) if c * lc // gc == b]
                bits[a, b], nats[a, b] = entropy(h[np.ix_(rows, cols)])
        out.append((bits, nats))
    return out


# --- gradient-based shuffle (Sections 5 and 8) ---------------------------------

def gradient_permutation(counts, stream_seed: int) -> np.ndarray:
    """G-R / G-C shuffle of n items with per-item nonzero counts h (row
    lengths, or column counts): the gradient g_i = h_{i+1} - h_i, the pivot
    p = first index of its maximum, the parts A = [0, p] and B = [p+1, n);
    each part is permuted at random (the stable order of the stream's keys
    restricted to that part) and the two are riffled like a deck of cards,
    A and B alternating and the longer part's remainder appended. Returns the
    new-to-old permutation."""
    h = np.asarray(counts, dtype=np.int64)
    n = len(h)
    if n < 2:
        return np.arange(n, dtype=np.int32)
    g = h[1:] - h[:-1]
    p = int(np.argmax(g))
    keys = splitmix64_outputs(stream_seed, n)
    A = np.arange(0, p + 1)
    B = np.arange(p + 1, n)
    A = A[np.argsort(keys[A], kind="stable")]
    B = B[np.argsort(keys[B], kind="stable")]
    m = min(len(A), len(B))
    out = np.empty(n, dtype=np.int64)
    out[0:2 * m:2] = A[:m]
    out[1:2 * m:2] = B[:m]
    out[2 * m:] = A[m:] if len(A) > m else B[m:]
    return out.astype(np.int32)


GRADIENT = 4


def permute_gradient(A, seed: int, mode: int = ROWS | GRADIENT):
    """Section 8's gradient formats: rows by the gradient shuffle when mode
    has ROWS (G-R), columns too when it has COLS (G-C). Returns
    (rperm, cperm, (rp, col, val))."""
    s_r, s_c = stream_seeds(seed)
    rperm = (gradient_permutation(A.row_lengths(), s_r) if mode & ROWS
             else np.arange(A.nrows, dtype=np.int32))
    cperm = (gradient_permutation(np.bincount(A.col, minlength=A.ncols), s_c) if mode & COLS
             else np.arange(A.ncols, dtype=np.int32))
    return rperm, cperm, permute_csr(A, rperm, cperm)


# --- SpMV / SpMM (Section 2) ------------------------------------------------

def spmm(nrows: int, row_ptr, col, val, X: np.ndarray) -> np.ndarray:
    """Y = A X in FP64, each y_i summed left to right over row i."""
    X = np.asarray(X, dtype=np.float64)
    k = 1 if X.ndim == 1 else X.shape[1]
    X2 = np.ascontiguousarray(X.reshape(len(X), k))
    Y = np.empty((nrows, k), dtype=np.float64)
    rp, c, v = _c_i32(row_ptr), _c_i32(col), _c_f64(val)
    _c().orc_spmm(nrows, _p(rp), _p(c), _p(v), k, _p(X2), k, _p(Y), k)
    return Y[:, 0].copy() if X.ndim == 1 else Y


def spmv(A, x):
    return spmm(A.nrows, A.row_ptr, A.col, A.val, x)


MIN_PLUS, OR_AND = 1, 2


def spmm_semiring(semiring: int, nrows: int, row_ptr, col, val, X: np.ndarray) -> np.ndarray:
    """Y = A X over (min, +) (semiring 1: y_i = min of val + x over row i's
    stored entries, +inf for an empty row) or (or, and) (semiring 2: y_i = 1
    if a stored nonzero meets a nonzero x, else 0), Section 2."""
    X = np.asarray(X, dtype=np.float64)
    k = 1 if X.ndim == 1 else X.shape[1]
    X2 = np.ascontiguousarray(X.reshape(len(X), k))
    Y = np.empty((nrows, k), dtype=np.float64)
    rp, c, v = _c_i32(row_ptr), _c_i32(col), _c_f64(val)
    fn = {MIN_PLUS: _c().orc_spmm_min_plus, OR_AND: _c().orc_spmm_or_and}[semiring]
    fn(nrows, _p(rp), _p(c), _p(v), k, _p(X2), k, _p(Y), k)
    return Y[:, 0].copy() if X.ndim == 1 else Y


def coo_rows(row_ptr) -> np.ndarray:
    """COO row index of every stored entry of a CSR matrix (Section 2: entry
    l of row i has ROW[l] = i), i.e. i repeated row_ptr[i+1] - row_ptr[i] times."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(rp) - 1, dtype=np.int32), np.diff(rp))


def coo_spmm(nrows: int, row, col, val, X: np.ndarray) -> np.ndarray:
    """Y = A X for A in COO form (any entry order, no duplicates required):
    Y = 0, then every entry in storage order adds val * X[col] to Y[row]."""
    X = np.asarray(X, dtype=np.float64)
    k = 1 if X.ndim == 1 else X.shape[1]
    X2 = np.ascontiguousarray(X.reshape(len(X), k))
    Y = np.empty((nrows, k), dtype=np.float64)
    r, c, v = _c_i32(row), _c_i32(col), _c_f64(val)
    _c().orc_coo_spmm(nrows, len(r), _p(r), _p(c), _p(v), k, _p(X2), k, _p(Y), k)
    return Y[:, 0].copy() if X.ndim == 1 else Y


def spmm_parallel(nrows: int, row_ptr, col, val, X: np.ndarray, Y: np.ndarray) -> None:
    """The same product on all OpenMP threads (equal-row static split).
    X, Y contiguous FP64 [n, k]; written in place."""
    k = 1 if X.ndim == 1 else X.shape[1]
    _c().orc_spmm_parallel(nrows, _p(row_ptr), _p(col), _p(val), k, _p(X), k, _p(Y), k)


def omp_threads() -> int:
    return int(_c().orc_omp_max_threads())


def permuted_spmm(A, rperm, cperm, B, X):
    """y = P_r^-1 ((P_r A P_c)(P_c^-1 x)) (Eq. 1), with B = (rp, col, val)
    the permuted matrix: gather x by cperm, multiply, scatter y by rperm."""
    X = np.asarray(X, dtype=np.float64)
    Xp = X[np.asarray(cperm, np.int64)]
    Yp = spmm(A.nrows, B[0], B[1], B[2], Xp)
    Y = np.empty_like(Yp)
    Y[np.asarray(rperm, np.int64)] = Yp
    return Y


# --- storage precision ------------------------------------------------------

def round_f32(vals) -> np.ndarray:
    v = _c_f64(vals)
    out = np.empty(len(v), np.float32)
    _c().orc_round_f32(len(v), _p(v), _p(out))
    return out


def round_bf16(vals) -> np.ndarray:
    """uint16 BF16 bit patterns, rounded once to nearest-even from FP64."""
    v = _c_f64(vals)
    out = np.empty(len(v), np.uint16)
    _c().orc_round_bf16(len(v), _p(v), _p(out))
    return out


def bf16_to_f64(bits) -> np.ndarray:
    """Exact value of BF16 bit patterns."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def stored_values(val, dtype: str) -> np.ndarray:
    """The FP64 value of what is stored for each entry."""
    if dtype == "f64":
        return _c_f64(val)
    if dtype == "f32":
        return round_f32(val).astype(np.float64)
    if dtype == "bf16":
        return bf16_to_f64(round_bf16(val))
    raise ValueError(dtype)


# --- error metric -----------------------------------------------------------

def normalized_error(nrows: int, row_ptr, col, val, X, Y, Yref) -> float:
    """max_i |y_i - yref_i| / (|A| |x|)_i over all rows and right-hand sides;
    a row whose (|A||x|)_i is zero must have y_i == 0 exactly, else the
    error is infinite."""
    X = np.asarray(X, dtype=np.float64)
    denom = spmm(nrows, row_ptr, col, np.abs(_c_f64(val)), np.abs(X))
    d = np.abs(np.asarray(Y, np.float64) - np.asarray(Yref, np.float64))
    zero = denom == 0
    if np.any(zero & (np.asarray(Y) != 0)):
        return float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(zero, 0.0, d / np.where(zero, 1.0, denom))
    return float(r.max()) if r.size else 0.0
