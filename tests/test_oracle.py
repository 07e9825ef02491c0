"""Pins for the CPU oracle: each check ties the oracle to something other than
itself (published known answers, independent libraries, closed forms, brute
force, invariants), chosen so a dropped term, a wrong index or a transposed
operand fails at least one of them. CPU only."""
import math
import os
from decimal import Decimal

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(A):
    D = np.zeros((A.nrows, A.ncols))
    for i in range(A.nrows):
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col[e]] = A.val[e]
    return D


def _scipy(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.nrows, A.ncols))


# --- keys ---------------------------------------------------------------------

def _golden_splitmix():
    outs, buckets = [], []
    with open(os.path.join(GOLDEN, "splitmix64_known_answers.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "outputs":
                outs.append((int(parts[1]), [int(v) for v in parts[2:]]))
            elif parts[0] == "buckets":
                buckets.append((int(parts[1]), int(parts[2]), [int(v) for v in parts[3:]]))
    return outs, buckets


def test_splitmix64_known_answers():
    outs, buckets = _golden_splitmix()
    assert outs and buckets
    for seed, expect in outs:
        assert oracle.splitmix64_outputs(seed, len(expect)).tolist() == expect
    for seed, n, counts in buckets:
        o = oracle.splitmix64_outputs(seed, n)
        u = (o >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        assert np.bincount(np.floor(u * 5).astype(int), minlength=5).tolist() == counts


def test_stream_seeds_are_first_two_outputs():
    for seed in (0, 3, 2**64 - 1):
        s_r, s_c = oracle.stream_seeds(seed)
        assert [s_r, s_c] == oracle.splitmix64_outputs(seed, 2).tolist()
        assert s_r != s_c


# --- permutations -------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2, 7, 4096, 100_003])
def test_permutation_bijection_and_inverse(n):
    s_r, _ = oracle.stream_seeds(3)
    p = oracle.permutation(n, s_r)
    assert p.dtype == np.int32 and len(p) == n
    assert np.array_equal(np.sort(p), np.arange(n))
    inv = oracle.inverse(p)
    assert np.array_equal(inv[p], np.arange(n))
    assert np.array_equal(p[inv], np.arange(n))


def test_permutation_is_library_stable_argsort_of_keys():
    s = oracle.stream_seeds(11)[1]
    n = 50_000
    keys = oracle.splitmix64_outputs(s, n)
    assert np.array_equal(oracle.permutation(n, s), np.argsort(keys, kind="stable"))


def test_argsort_ties_keep_index_order():
    keys = np.array([5, 3, 5, 3, 1, 5], dtype=np.uint64)
    perm = np.empty(6, np.int32)
    oracle._c().orc_argsort_keys(6, oracle._p(keys), oracle._p(perm))
    assert perm.tolist() == [4, 1, 3, 0, 2, 5]


def test_permutation_uniform_over_s4():
    """All 24 permutations of 4 items appear equally often over many seeds
    (chi-square, 23 degrees of freedom)."""
    counts = {}
    trials = 24_000
    for seed in range(trials):
        p = tuple(oracle.permutation(4, oracle.stream_seeds(seed)[0]).tolist())
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == 24
    obs = np.array(list(counts.values()))
    chi2 = ((obs - trials / 24) ** 2 / (trials / 24)).sum()
    assert scipy.stats.chi2.sf(chi2, 23) > 1e-4


# --- permuted CSR ---------------------------------------------------------------

@pytest.mark.parametrize("shape,density,seed", [((1, 1), 1.0, 0), ((37, 53), 0.2, 1),
                                                ((64, 64), 0.05, 2), ((200, 90), 0.1, 3)])
def test_permute_csr_matches_scipy_slicing(shape, density, seed):
    A = synth.random_csr(shape[0], shape[1], density, seed, empty_rows=0.2)
    rperm, cperm, (rp, col, val) = oracle.permute(A, seed + 100)
    S = _scipy(A)[rperm][:, cperm].tocsr()
    S.sort_indices()
    assert np.array_equal(rp, S.indptr)
    assert np.array_equal(col, S.indices)
    assert np.array_equal(val, S.data)          # values move bit-exact


def test_permute_csr_dense_brute_force_and_modes():
    A = synth.random_csr(23, 31, 0.3, 5)
    D = _dense(A)
    for mode in (oracle.ROWS, oracle.COLS, oracle.ROWS | oracle.COLS):
        rperm, cperm, (rp, col, val) = oracle.permute(A, 9, mode)
        if not mode & oracle.ROWS:
            assert np.array_equal(rperm, np.arange(23))
        if not mode & oracle.COLS:
            assert np.array_equal(cperm, np.arange(31))
        B = synth.CSR(23, 31, rp, col, val)
        Dp = np.zeros_like(D)
        for i in range(23):             # B[i, j] = A[rperm[i], cperm[j]]
            for j in range(31):
                Dp[i, j] = D[rperm[i], cperm[j]]
        assert np.array_equal(_dense(B), Dp)
        for i in range(23):             # canonical: strictly increasing columns
            assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)


def test_permute_same_seed_same_result():
    A = synth.random_csr(50, 50, 0.1, 7)
    r1 = oracle.permute(A, 42)
    r2 = oracle.permute(A, 42)
    for a, b in zip(r1[:2] + r1[2], r2[:2] + r2[2]):
        assert np.array_equal(a, b)
    r3 = oracle.permute(A, 43)
    assert not np.array_equal(r1[0], r3[0])


# --- histogram ------------------------------------------------------------------

def _hist_by_edges(A, gr, gc):
    """Same histogram by another route: block b starts at the first index t
    with t*G >= b*M, i.e. ceil(b*M/G); counted with numpy's histogram2d."""
    rows = np.repeat(np.arange(A.nrows), A.row_lengths())
    er = np.array([-(-b * A.nrows // gr) for b in range(gr + 1)], dtype=np.float64) - 0.5
    ec = np.array([-(-b * A.ncols // gc) for b in range(gc + 1)], dtype=np.float64) - 0.5
    h, _, _ = np.histogram2d(rows, A.col, bins=[er, ec])
    return h.astype(np.int64)


@pytest.mark.parametrize("m,n,gr,gc", [(64, 64, 8, 8), (100, 37, 7, 3), (37, 100, 3, 7),
                                       (10, 10, 10, 10), (5, 9, 16, 4), (1000, 1000, 64, 64)])
def test_block_hist_by_edges_and_sum(m, n, gr, gc):
    A = synth.random_csr(m, n, 0.2, m + n)
    h = oracle.block_hist(A.nrows, A.ncols, A.row_ptr, A.col, gr, gc)
    assert h.shape == (gr, gc)
    assert h.sum() == A.nnz
    if gr <= m and gc <= n:
        assert np.array_equal(h, _hist_by_edges(A, gr, gc))


def test_block_hist_rows_per_block_differ_by_at_most_one():
    m, g = 2_000_003, 1024
    A = synth.CSR(m, 1, np.arange(m + 1, dtype=np.int32), np.zeros(m, np.int32), np.ones(m))
    h = oracle.block_hist(m, 1, A.row_ptr, A.col, g, 1)[:, 0]
    assert h.sum() == m and h.max() - h.min() <= 1 and h.min() == m // g


def test_block_hist_transposed_shape_distinguished():
    A = synth.random_csr(30, 12, 0.5, 1)
    h = oracle.block_hist(30, 12, A.row_ptr, A.col, 5, 2)
    rows = np.repeat(np.arange(30), A.row_lengths())
    brute = np.zeros((5, 2), np.int64)
    for r, c in zip(rows, A.col):
        brute[r // 6, c // 6] += 1        # 30/5 = 6 rows and 12/2 = 6 columns per block
    assert np.array_equal(h, brute)


def test_block_hist_uniform_fill():
    U = synth.uniform_fill(4096, 64, 16)
    h = oracle.block_hist(U.nrows, U.ncols, U.row_ptr, U.col, 64, 64)
    assert np.all(h == 16)


def test_block_hist_of_permuted_equals_remapped_entries():
    A = synth.random_csr(300, 200, 0.05, 4)
    rperm, cperm, (rp, col, val) = oracle.permute(A, 5)
    rinv, cinv = oracle.inverse(rperm), oracle.inverse(cperm)
    rows = np.repeat(np.arange(300), A.row_lengths())
    # entry (i, j) of A sits at (rinv[i], cinv[j]) in B
    nr, nc = rinv[rows], cinv[A.col]
    brute = np.zeros((16, 8), np.int64)
    np.add.at(brute, (nr * 16 // 300, nc * 8 // 200), 1)
    assert np.array_equal(oracle.block_hist(300, 200, rp, col, 16, 8), brute)


# --- entropy --------------------------------------------------------------------

def test_entropy_closed_forms():
    assert oracle.entropy([0, 0, 7, 0]) == (0.0, 0.0)        # one bin: no uncertainty
    assert oracle.entropy([]) == (0.0, 0.0)
    assert oracle.entropy([0, 0]) == (0.0, 0.0)
    bits, nats = oracle.entropy(np.full(4096, 16))
    assert bits == 12.0
    assert nats == pytest.approx(12 * math.log(2), rel=1e-15)
    # uniform over 3 bins: log2 3 and ln 3, from their published decimal
    # expansions (OEIS A020857 and A002391) rounded once to double
    bits, nats = oracle.entropy([5, 5, 5])
    assert bits == float(Decimal("1.58496250072115618145373894394781650875981440769"))
    assert nats == float(Decimal("1.09861228866810969139524523692252570464749055782"))
    bits, _ = oracle.entropy([1, 0, 3])                       # 2 - (3/4) log2 3
    assert bits == pytest.approx(2 - 0.75 * math.log2(3), rel=0, abs=4e-16)
    bits, _ = oracle.entropy([1, 1])
    assert bits == 1.0


def test_entropy_matches_scipy_and_bounds():
    rng = np.random.default_rng(0)
    for trial in range(5):
        h = rng.poisson(rng.uniform(0.5, 30), size=rng.integers(2, 5000))
        if h.sum() == 0:
            continue
        bits, nats = oracle.entropy(h)
        assert bits == pytest.approx(scipy.stats.entropy(h, base=2), rel=1e-12)
        assert nats == pytest.approx(scipy.stats.entropy(h), rel=1e-12)
        assert bits <= math.log2(len(h))
        # order of the bins does not matter (Section 5)
        assert oracle.entropy(rng.permutation(h)) == (bits, nats)


def test_entropy_uniform_fill_matrix_reaches_log_blocks():
    U = synth.uniform_fill(4096, 64, 16)
    h = oracle.block_hist(U.nrows, U.ncols, U.row_ptr, U.col, 64, 64)
    assert oracle.entropy(h)[0] == 12.0


def test_entropy_rises_after_permutation():
    """Sanity: the block-clustered matrix's entropy rises towards log2(4096)
    once permuted (analytic expectation for a random placement of S entries
    in B bins: log2 B - (B-1)/(2 S ln 2) to first order)."""
    A = synth.clustered_n4096(1)
    h0 = oracle.block_hist(A.nrows, A.ncols, A.row_ptr, A.col, 64, 64)
    _, _, (rp, col, _) = oracle.permute(A, 3)
    h1 = oracle.block_hist(A.nrows, A.ncols, rp, col, 64, 64)
    H0, H1 = oracle.entropy(h0)[0], oracle.entropy(h1)[0]
    expect = 12 - 4095 / (2 * A.nnz * math.log(2))
    assert H0 < 8.5
    assert abs(H1 - expect) < 0.01


# --- SpMV / SpMM ----------------------------------------------------------------

def test_spmv_bit_exact_vs_dense_brute_force():
    A = synth.random_csr(40, 33, 0.3, 8, empty_rows=0.2)
    D = _dense(A)
    x = synth.vector(33, 9)
    y = oracle.spmv(A, x)
    for i in range(40):
        acc = 0.0
        for j in range(33):             # increasing j, zeros included
            acc += D[i, j] * x[j]
        assert y[i] == acc


def test_spmm_columns_equal_spmv_and_scipy():
    A = synth.random_csr(120, 90, 0.08, 10)
    X = synth.vector(90, 11, k=5)
    Y = oracle.spmm(A.nrows, A.row_ptr, A.col, A.val, X)
    for c in range(5):
        assert np.array_equal(Y[:, c], oracle.spmv(A, np.ascontiguousarray(X[:, c])))
    ref = _scipy(A) @ X
    err = oracle.normalized_error(A.nrows, A.row_ptr, A.col, A.val, X, Y, ref)
    assert err < 1e-15


def test_coo_rows_expand_row_ptr():
    rp = np.array([0, 2, 2, 5, 6], np.int32)
    assert oracle.coo_rows(rp).tolist() == [0, 0, 2, 2, 2, 3]
    assert oracle.coo_rows(np.array([0], np.int32)).tolist() == []


def test_coo_spmv_dense_brute_force_and_scipy():
    A = synth.random_csr(40, 33, 0.3, 8, empty_rows=0.2)
    D = _dense(A)
    x = synth.vector(33, 9)
    row = oracle.coo_rows(A.row_ptr)
    y = oracle.coo_spmm(A.nrows, row, A.col, A.val, x)
    for i in range(40):                 # sorted COO: each row's terms in increasing column
        acc = 0.0
        for j in range(33):
            acc += D[i, j] * x[j]
        assert y[i] == acc
    # entries in any order: the same matrix, within rounding of scipy's COO product
    import scipy.sparse as sp
    perm = np.random.default_rng(3).permutation(A.nnz)
    X = synth.vector(33, 10, k=3)
    Y = oracle.coo_spmm(A.nrows, row[perm], A.col[perm], A.val[perm], X)
    ref = sp.coo_matrix((A.val[perm], (row[perm], A.col[perm])), shape=(40, 33)) @ X
    assert oracle.normalized_error(A.nrows, A.row_ptr, A.col, A.val, X, Y, ref) < 1e-15
    assert np.all(Y[np.diff(A.row_ptr) == 0] == 0.0)   # empty rows are exactly zero


def test_semiring_products_dense_brute_force():
    A = synth.random_csr(30, 25, 0.2, 14, empty_rows=0.2)
    X = synth.vector(25, 15, k=2)
    X[3] = 0.0                                       # zeros in x matter for (or, and)
    Amp = oracle.spmm_semiring(oracle.MIN_PLUS, A.nrows, A.row_ptr, A.col, A.val, X)
    Aor = oracle.spmm_semiring(oracle.OR_AND, A.nrows, A.row_ptr, A.col, A.val, X)
    for i in range(A.nrows):
        cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        vals = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        for c in range(2):
            terms = [v + X[j, c] for j, v in zip(cols, vals)]
            assert Amp[i, c] == (min(terms) if terms else np.inf)
            assert Aor[i, c] == float(any(v != 0 and X[j, c] != 0 for j, v in zip(cols, vals)))


def test_min_plus_iteration_gives_shortest_paths():
    """Bellman-Ford as repeated (min, +) products with the transposed weight
    matrix equals scipy's shortest paths; integer weights keep sums exact."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(4)
    n = 60
    W = synth.random_csr(n, n, 0.06, 16)
    W.val = rng.integers(1, 10, size=W.nnz).astype(np.float64)
    Wt = sp.csr_matrix((W.val, W.col, W.row_ptr), shape=(n, n)).T.tocsr()
    Wt.sort_indices()
    for s0 in (0, 7):
        d = np.full(n, np.inf)
        d[s0] = 0.0
        for _ in range(n - 1):
            d = np.minimum(d, oracle.spmm_semiring(oracle.MIN_PLUS, n, Wt.indptr, Wt.indices,
                                                   Wt.data, d))
        ref = shortest_path(sp.csr_matrix((W.val, W.col, W.row_ptr), shape=(n, n)),
                            directed=True, indices=s0)
        assert np.array_equal(d, ref)


def test_or_and_iteration_gives_reachability():
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order
    n = 80
    W = synth.random_csr(n, n, 0.025, 17)
    Wt = sp.csr_matrix((W.val, W.col, W.row_ptr), shape=(n, n)).T.tocsr()
    Wt.sort_indices()
    for s0 in (0, 11):
        r = np.zeros(n)
        r[s0] = 1.0
        for _ in range(n):
            r = np.maximum(r, oracle.spmm_semiring(oracle.OR_AND, n, Wt.indptr, Wt.indices,
                                                   Wt.data, r))
        order = breadth_first_order(sp.csr_matrix((W.val, W.col, W.row_ptr), shape=(n, n)), s0,
                                    directed=True, return_predecessors=False)
        assert set(np.nonzero(r)[0].tolist()) == set(order.tolist())


def test_spmm_parallel_equals_serial():
    A = synth.random_csr(500, 300, 0.05, 12)
    X = np.ascontiguousarray(synth.vector(300, 13, k=3))
    Y = np.empty((500, 3))
    oracle.spmm_parallel(A.nrows, A.row_ptr, A.col, A.val, X, Y)
    assert np.array_equal(Y, oracle.spmm(A.nrows, A.row_ptr, A.col, A.val, X))


def test_permuted_product_identity():
    """y = P_r^-1 ((P_r A P_c)(P_c^-1 x)) equals A x (Eq. 1)."""
    A = synth.clustered_n4096(1)
    x = synth.vector(A.ncols, 2)
    rperm, cperm, B = oracle.permute(A, 3)
    y = oracle.permuted_spmm(A, rperm, cperm, B, x)
    ref = oracle.spmv(A, x)
    assert oracle.normalized_error(A.nrows, A.row_ptr, A.col, A.val, x, y, ref) < 1e-15


# --- storage precision ----------------------------------------------------------

def _golden_bf16():
    cases = []
    with open(os.path.join(GOLDEN, "bf16_rounding_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            expr, rest = line.split("0x", 1)
            cases.append((float(eval(expr, {"__builtins__": {}})), int(rest.split()[0], 16)))
    return cases


def test_bf16_halfway_cases():
    cases = _golden_bf16()
    assert len(cases) >= 10
    for v, bits in cases:
        assert int(oracle._c().orc_bf16_from_f64(v)) == bits, (v, hex(bits))


def test_bf16_matches_torch_on_fp32_exact_inputs():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    v32 = np.concatenate([rng.uniform(-1, 1, 20000), rng.standard_normal(20000) * 1e30,
                          rng.standard_normal(2000) * 1e-39]).astype(np.float32)
    ref = torch.from_numpy(v32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.round_bf16(v32.astype(np.float64)), ref)


def _golden_bf16_decode():
    cases = []
    with open(os.path.join(GOLDEN, "bf16_decode_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            bits, rest = line.split(None, 1)
            expr = rest.split("  ")[0].strip()
            val = float(expr) if expr in ("inf", "-inf") else float(eval(expr, {"__builtins__": {}}))
            cases.append((int(bits, 16), val))
    return cases


def test_bf16_to_f64_hand_decoded_patterns():
    """The oracle's BF16 decode gives the exact values worked out by hand from
    the bit layout (sign, exponent bias, subnormals, infinities)."""
    cases = _golden_bf16_decode()
    assert len(cases) >= 12
    got = oracle.bf16_to_f64(np.array([b for b, _ in cases], np.uint16))
    for (bits, want), g in zip(cases, got):
        assert g == want and math.copysign(1.0, g) == math.copysign(1.0, want), (hex(bits), g, want)
    assert np.isnan(oracle.bf16_to_f64(np.array([0x7FC0, 0xFFC1], np.uint16))).all()


def test_bf16_to_f64_matches_torch_on_every_pattern():
    """All 65536 BF16 patterns decode to torch's bfloat16 -> float64 value."""
    torch = pytest.importorskip("torch")
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    with np.errstate(invalid="ignore"):              # signalling NaN patterns
        got = oracle.bf16_to_f64(bits)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint64), ref[~nan].view(np.uint64))


def test_stored_values_per_storage():
    """What the GPU stores, as FP64: the value itself (FP64), numpy's IEEE
    rounding to float32 (FP32), and for BF16 the golden rounding cases decoded
    by Python's own binary32 unpacking, plus torch's rounding on FP32-exact
    inputs."""
    import struct
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.uniform(-1, 1, 5000), rng.standard_normal(5000) * 1e20])
    assert np.array_equal(oracle.stored_values(v, "f64").view(np.uint64), v.view(np.uint64))
    f32 = oracle.stored_values(v, "f32")
    assert np.array_equal(f32.view(np.uint64), v.astype(np.float32).astype(np.float64).view(np.uint64))
    for x, bits in _golden_bf16():
        want = struct.unpack(">f", struct.pack(">I", bits << 16))[0]
        got = float(oracle.stored_values(np.array([x]), "bf16")[0])
        assert got == want and math.copysign(1.0, got) == math.copysign(1.0, want), (x, hex(bits))
    torch = pytest.importorskip("torch")
    v32 = v.astype(np.float32)
    ref = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.stored_values(v32.astype(np.float64), "bf16"), ref)
    with pytest.raises(ValueError):
        oracle.stored_values(v, "f16")


def test_f32_rounding_matches_numpy_and_nan_bf16():
    v = np.random.default_rng(2).uniform(-1, 1, 10000)
    assert np.array_equal(oracle.round_f32(v), v.astype(np.float32))
    assert int(oracle._c().orc_bf16_from_f64(float("nan"))) & 0x7F80 == 0x7F80
    assert int(oracle._c().orc_bf16_from_f64(float("inf"))) == 0x7F80
    assert int(oracle._c().orc_bf16_from_f64(-1e300)) == 0xFF80


def test_normalized_error_hand_cases():
    A = synth.CSR(3, 2, np.array([0, 2, 2, 3], np.int32), np.array([0, 1, 1], np.int32),
                  np.array([1.0, -2.0, 4.0]))
    x = np.array([1.0, 0.5])
    ref = np.array([0.0, 0.0, 2.0])
    assert oracle.normalized_error(3, A.row_ptr, A.col, A.val, x, ref, ref) == 0.0
    y = np.array([1e-3, 0.0, 2.0])      # |A||x| row 0 = 1 + 1 = 2
    assert oracle.normalized_error(3, A.row_ptr, A.col, A.val, x, y, ref) == pytest.approx(5e-4)
    y = np.array([0.0, 1e-300, 2.0])    # empty row must be exactly zero
    assert oracle.normalized_error(3, A.row_ptr, A.col, A.val, x, y, ref) == float("inf")


# --- hierarchical entropy (Section 5) ---------------------------------------------

def test_entropy_levels_uniform_and_global():
    h = np.full((64, 64), 16)
    lv = oracle.entropy_levels(h, levels=(1, 2, 4, 8))
    assert lv[0][0][0, 0] == oracle.entropy(h)[0] == 12.0       # one region: the global H
    for (bits, _), expect in zip(lv[1:], (10.0, 8.0, 6.0)):     # 32x32, 16x16, 8x8 bins each
        assert np.all(bits == expect)


def test_entropy_levels_hand_cases():
    h = np.array([[1, 0], [0, 3]])
    (bits, nats), = oracle.entropy_levels(h, levels=(2,))
    assert np.all(bits == 0.0) and np.all(nats == 0.0)          # one nonzero bin per region
    h = np.array([[1, 1, 0, 4], [2, 2, 0, 0]])
    (bits, _), = oracle.entropy_levels(h, levels=(2,))
    assert bits.shape == (2, 2)
    assert bits[0, 0] == 1.0 and bits[1, 0] == 1.0                # two equal bins
    assert bits[0, 1] == 0.0 and bits[1, 1] == 0.0
    (bits, _), = oracle.entropy_levels(np.ones((3, 5), np.int64), levels=(4,))
    assert bits.shape == (3, 4)                                    # fewer regions than L rows


# --- gradient shuffle (Sections 5 and 8) -------------------------------------------

def test_gradient_permutation_structure():
    h = np.array([1, 1, 1, 9, 9, 9, 9, 9, 2])     # steepest rise between rows 2 and 3
    s = oracle.stream_seeds(5)[0]
    p = oracle.gradient_permutation(h, s)
    assert sorted(p.tolist()) == list(range(9))
    A, B = {0, 1, 2}, {3, 4, 5, 6, 7, 8}
    # riffle: A and B alternate while both last, then B's remainder
    assert [int(v) in A for v in p[:6:2]] == [True] * 3
    assert all(int(v) in B for v in p[1:6:2]) and all(int(v) in B for v in p[6:])
    keys = oracle.splitmix64_outputs(s, 9)
    a_order = [int(v) for v in p if int(v) in A]
    b_order = [int(v) for v in p if int(v) in B]
    assert a_order == sorted(A, key=lambda i: (keys[i], i))       # random order inside each part
    assert b_order == sorted(B, key=lambda i: (keys[i], i))


def test_gradient_permutation_edges():
    s = oracle.stream_seeds(1)[0]
    assert oracle.gradient_permutation([], s).tolist() == []
    assert oracle.gradient_permutation([7], s).tolist() == [0]
    p = oracle.gradient_permutation([5, 5, 5], s)                  # ties: first index, p = 0
    assert p[0] == 0 and sorted(p[1:].tolist()) == [1, 2]
    p = oracle.gradient_permutation([3, 2, 1, 0], s)              # all falling: max gradient -1 at 0
    assert p[0] == 0
    for n in (2, 17, 1000):
        h = np.random.default_rng(n).integers(0, 50, size=n)
        q = oracle.gradient_permutation(h, s)
        assert np.array_equal(np.sort(q), np.arange(n))


def test_permute_gradient_modes():
    A = synth.random_csr(40, 30, 0.2, 3)
    rperm, cperm, (rp, col, val) = oracle.permute_gradient(A, 7, oracle.ROWS | oracle.GRADIENT)
    assert np.array_equal(cperm, np.arange(30))
    s_r, s_c = oracle.stream_seeds(7)
    assert np.array_equal(rperm, oracle.gradient_permutation(A.row_lengths(), s_r))
    rperm, cperm, _ = oracle.permute_gradient(A, 7, oracle.ROWS | oracle.COLS | oracle.GRADIENT)
    assert np.array_equal(cperm, oracle.gradient_permutation(np.bincount(A.col, minlength=30), s_c))
    S = _scipy(A)[rperm][:, cperm].tocsr()
    S.sort_indices()
    _, _, (rp, col, val) = oracle.permute_gradient(A, 7, oracle.ROWS | oracle.COLS | oracle.GRADIENT)
    assert np.array_equal(rp, S.indptr) and np.array_equal(col, S.indices)
