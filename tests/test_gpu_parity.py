"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer results (permutations, permuted CSR, histograms) and the correctly
rounded entropy must match bit for bit; products must stay within
max_i |y - y_ref| / (|A||x|)_i of 1e-13 (FP64), 1e-5 (FP32 values) and 1e-2
(BF16 values, FP32 accumulation) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL, expected_export, spmv_error, torch_vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mx = pytest.importorskip("paper_2308_00106_amd.mxe")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mx.Context(0)
    yield c
    c.close()


def _diag(n, m=None):
    m = n if m is None else m
    k = min(n, m)
    rp = np.concatenate([np.arange(k + 1), np.full(n - k, k)]).astype(np.int32)
    return synth.CSR(n, m, rp, np.arange(k, dtype=np.int32), np.ones(k))


# --- permutations -------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 48, 49, 50, 1000, 4096, 100_003, 2_000_000])
def test_permutation_matches_oracle(ctx, n):
    m = max(1, n // 3 + 5)
    A = ctx.register(_diag(n, m))
    for seed in (3, 0, 2**64 - 1):
        B = ctx.permute(A, seed)
        rp, cp = ctx.get_permutation(B)
        s_r, s_c = oracle.stream_seeds(seed)
        assert np.array_equal(rp, oracle.permutation(n, s_r)), (n, seed)
        assert np.array_equal(cp, oracle.permutation(m, s_c)), (n, seed)
        ctx.release(B)
    ctx.release(A)


@pytest.mark.slow
@pytest.mark.parametrize("n", [9_000_000, 40_000_000])
def test_permutation_large_n_bucket_path(ctx, n):
    """Above 2048 << 12 indices the permutation buckets with device atomics
    (up to 2^20 buckets of ~2K) before the same per-bucket LDS sort."""
    A = ctx.register(_diag(n, 7))
    B = ctx.permute(A, 5, mx.ROWS)
    rp, _ = ctx.get_permutation(B)
    assert np.array_equal(rp, oracle.permutation(n, oracle.stream_seeds(5)[0]))
    ctx.release(B)
    ctx.release(A)


def test_permute_modes_identity_parts(ctx):
    A0 = synth.random_csr(300, 200, 0.05, 1)
    A = ctx.register(A0)
    B = ctx.permute(A, 9, mx.ROWS)
    rp, cp = ctx.get_permutation(B)
    assert np.array_equal(cp, np.arange(200))
    assert np.array_equal(rp, oracle.permute(A0, 9, oracle.ROWS)[0])
    C = ctx.permute(A, 9, mx.COLS)
    rp, cp = ctx.get_permutation(C)
    assert np.array_equal(rp, np.arange(300))
    assert np.array_equal(cp, oracle.permute(A0, 9, oracle.COLS)[1])
    for H in (B, C, A):
        ctx.release(H)


# --- permuted CSR ---------------------------------------------------------------

CSR_CASES = [
    ("clustered_n4096", lambda: synth.clustered_n4096(1)),
    ("ragged", lambda: synth.random_csr(4096 * 3 + 17, 9001, 0.002, 2, empty_rows=0.1)),
    ("wide", lambda: synth.random_csr(333, 20000, 0.01, 3)),
    # ~450 entries per row: groups of rows exceed the 1024-entry LDS stage, so
    # rows move one at a time, each staged in LDS
    ("long_rows", lambda: synth.random_csr(700, 3000, 0.15, 4)),
    # rows of 1025-8000 entries (columns 1M, so no row is dense): longer than
    # the stage, each entry is ranked against cinv in global memory
    ("rows_over_1024", lambda: synth.block_clustered(
        48, np.random.default_rng(6).integers(1025, 8001, size=48), 4096, 0.1, 6, ncols=1_000_000)),
    ("empty", lambda: synth.random_csr(50, 60, 0.0, 5)),
    ("skewed", lambda: synth.skewed_n4m(1, n=60_000)),
]


@pytest.mark.parametrize("name,make", CSR_CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_permuted_csr_bit_exact(ctx, name, make, storage):
    A0 = make()
    A = ctx.register(A0, storage)
    for mode in (mx.ROWS | mx.COLS, mx.ROWS, mx.COLS):
        B = ctx.permute(A, 3, mode)
        rperm, cperm = ctx.get_permutation(B)
        er, ec, ev = expected_export(A0, rperm, cperm, storage)
        gr, gc, gv = ctx.export_csr(B)
        assert np.array_equal(gr, er), (name, mode)
        assert np.array_equal(gc, ec), (name, mode)
        assert np.array_equal(gv.view(np.uint8), np.asarray(ev).view(np.uint8)), (name, mode)
        ctx.release(B)
    ctx.release(A)


def test_registered_values_round_once(ctx):
    """BF16/FP32 storage equals one round-to-nearest-even from FP64."""
    vals = np.array([1 + 2**-8 + 2**-30, 1 + 2**-8, 1 + 3 * 2**-8, -(2 - 2**-8) * 2.0**127,
                     1.5 * 2.0**-133, 2.0**-126 - 2.0**-134, 0.1, -0.0, 3.0e38, 1e-45])
    n = len(vals)
    A0 = synth.CSR(1, n, np.array([0, n], np.int32), np.arange(n, dtype=np.int32), vals)
    for storage, ref in (("bf16", oracle.round_bf16(vals)), ("f32", oracle.round_f32(vals))):
        A = ctx.register(A0, storage)
        _, _, gv = ctx.export_csr(A)
        assert np.array_equal(gv.view(np.uint8), ref.view(np.uint8)), storage
        ctx.release(A)


# --- histogram and entropy -----------------------------------------------------

@pytest.mark.parametrize("case,grid", [("clustered_n4096", (64, 64)), ("clustered_n4096", (1, 1)),
                                       ("clustered_n4096", (7, 3)), ("clustered_n4096", (4096, 1)),
                                       ("ragged", (64, 64)), ("wide", (5, 1000)),
                                       ("skewed", (1024, 1024)), ("skewed", (3, 20000))])
def test_histogram_and_entropy_exact(ctx, case, grid):
    A0 = dict(CSR_CASES)[case]()
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    for H in (A, B):
        rp, col, _ = ctx.export_csr(H)
        bits, nats, hist = ctx.entropy(H, grid[0], grid[1], hist=True)
        ref = oracle.block_hist(A0.nrows, A0.ncols, rp, col, grid[0], grid[1])
        assert np.array_equal(hist, ref), case
        assert (bits, nats) == oracle.entropy(ref), case
    ctx.release(B)
    ctx.release(A)


def test_entropy_uniform_fill_and_single_block(ctx):
    U = ctx.register(synth.uniform_fill(4096, 64, 16))
    assert ctx.entropy(U, 64, 64)[0] == 12.0
    assert ctx.entropy(U, 1, 1) == (0.0, 0.0)
    ctx.release(U)
    E = ctx.register(synth.random_csr(10, 10, 0.0, 1))
    assert ctx.entropy(E, 4, 4) == (0.0, 0.0)
    ctx.release(E)


def test_entropy_permuted_clustered_n4096(ctx):
    A0 = synth.clustered_n4096(1)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    h0, h1 = ctx.entropy(A, 64, 64)[0], ctx.entropy(B, 64, 64)[0]
    assert h0 < h1 <= 12.0
    ctx.release(B)
    ctx.release(A)


def test_entropy_rejects_bad_grid(ctx):
    A = ctx.register(synth.clustered_n4096(1))
    for g in ((0, 4), (4, 0), (2**20 + 1, 1)):
        with pytest.raises(mx.MxeError) as e:
            ctx.entropy(A, *g)
        assert e.value.status == mx.ERR_INVALID_ARG
    ctx.release(A)


# --- products -------------------------------------------------------------------

VARIANTS = [mx.variant(mx.VAR_GROUP, lanes) for lanes in (1, 2, 4, 8, 16, 32, 64)] + \
           [mx.variant(mx.VAR_BINNED), mx.variant(mx.VAR_MERGE),
            mx.variant(mx.VAR_SLAB, 1), mx.variant(mx.VAR_SLAB, 32),   # 64 KiB and 2 MiB slabs
            mx.variant(mx.VAR_SLAB, 16 | mx.SLAB_ONE_PER_CU),          # row blocks for one per CU
            mx.variant(mx.VAR_FIXED, 4), mx.variant(mx.VAR_FIXED, 16), mx.variant(mx.VAR_COO),
            # the slab layouts plus an LDS window of x per row block: one and two
            # workgroups per CU, and 64 KiB slabs (many slabs around the window)
            mx.variant(mx.VAR_WINDOW, 16 | mx.SLAB_ONE_PER_CU), mx.variant(mx.VAR_WINDOW, 32),
            mx.variant(mx.VAR_WINDOW, 1)]


def _force(ctx, H, k, v):
    """Forces variant v for every column chunk of a k-column product; False
    when the library declines it for this matrix (e.g. too many slabs)."""
    try:
        ctx.set_variant(H, min(k, 16), v)
        if k > 16:
            ctx.set_variant(H, k - 16, v)
    except mx.MxeError as e:
        if e.status == mx.ERR_UNSUPPORTED:
            return False
        raise
    return True


@pytest.mark.parametrize("name,make", CSR_CASES)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 8, 16, 17])
def test_spmv_all_variants_f64(ctx, name, make, k):
    A0 = make()
    X = synth.vector(A0.ncols, 2, k=k)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    rperm, cperm = ctx.get_permutation(B)
    Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
    for H, Ho in ((A, A0), (B, Bo)):
        Xt = torch_vec(X, torch.float64)
        for v in VARIANTS:
            if not _force(ctx, H, k, v):
                continue
            Y = torch.full((A0.nrows, k) if k > 1 else (A0.nrows,), float("nan"),
                           dtype=torch.float64, device="cuda")
            ctx.spmv(H, Xt, Y)
            torch.cuda.synchronize()
            err = spmv_error(Ho, X, Y.cpu().numpy(), "f64")
            assert err <= TOL["f64"], (name, k, hex(v), err)
    ctx.release(B)
    ctx.release(A)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("name,make", CSR_CASES[:4] + CSR_CASES[5:])
def test_spmv_reduced_precision(ctx, storage, name, make):
    A0 = make()
    for k in (1, 2, 4, 8, 12, 16):
        X = synth.vector(A0.ncols, 2, k=k)
        A = ctx.register(A0, storage)
        Xt = torch_vec(X, torch.float32)
        for v in VARIANTS:
            if not _force(ctx, A, k, v):
                continue
            Y = torch.full((A0.nrows, k) if k > 1 else (A0.nrows,), float("nan"),
                           dtype=torch.float32, device="cuda")
            ctx.spmv(A, Xt, Y)
            torch.cuda.synchronize()
            Yh = Y.cpu().numpy().astype(np.float64)
            err = spmv_error(A0, X, Yh, storage)           # vs FP64 oracle, original values
            assert err <= TOL[storage], (name, storage, k, hex(v), err)
        ctx.release(A)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_slab_x_rows_vector_or_scalar(ctx, storage):
    """The slab kernel reads an X row as vectors of min(16, k x 4 or 8) bytes
    only when k fills its class and the rows are aligned to that width, else
    element by element: both ways, on the permuted and the original matrix,
    for leading dimensions k (aligned), k + 1 and k + 2 (aligned or not)."""
    import torch
    A0 = synth.clustered_n4096(1)
    A = ctx.register(A0, storage)
    B = ctx.permute(A, 9)
    rperm, cperm = ctx.get_permutation(B)
    Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
    dt = torch.float64 if storage == "f64" else torch.float32
    tol = TOL["f64"] if storage == "f64" else TOL["f32"]     # against the stored values
    for H, Ho in ((A, A0), (B, Bo)):
        for k in (2, 4, 8):
            for v in (mx.variant(mx.VAR_SLAB, 16), mx.variant(mx.VAR_WINDOW, 32)):
                if not _force(ctx, H, k, v):
                    continue
                for ld in (k, k + 1, k + 2):
                    X = synth.vector(A0.ncols, 20 + ld, k=k)
                    Xf = X.astype(np.float32).astype(np.float64) if storage != "f64" else X
                    Xs = torch.zeros((A0.ncols, ld), dtype=dt, device="cuda")
                    Xs[:, :k] = torch_vec(Xf, dt)
                    Y = torch.full((A0.nrows, k), float("nan"), dtype=dt, device="cuda")
                    ctx.spmv(H, Xs[:, :k], Y)
                    torch.cuda.synchronize()
                    err = spmv_error(Ho, Xf, Y.cpu().numpy().astype(np.float64), storage,
                                     ref_stored=True)
                    assert err <= tol, (storage, k, ld, hex(v), err)
    ctx.release(B)
    ctx.release(A)


def test_identity_original_space(ctx):
    """y = P_r^-1 ((P_r A P_c)(P_c^-1 x)) equals A x (Eq. 1), via the
    original-space flag and via explicit gather / scatter."""
    A0 = synth.clustered_n4096(1)
    x = synth.vector(A0.ncols, 2)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    xt = torch_vec(x, torch.float64)
    y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
    ctx.spmv(B, xt, y, flags=mx.SPACE_ORIGINAL)
    torch.cuda.synchronize()
    assert spmv_error(A0, x, y.cpu().numpy(), "f64") <= 1e-13
    xp = torch.empty_like(xt)
    yp = torch.empty_like(y)
    y2 = torch.empty_like(y)
    ctx.gather_x(B, xt, xp)
    ctx.spmv(B, xp, yp)
    ctx.scatter_y(B, yp, y2)
    torch.cuda.synchronize()
    _, cperm = ctx.get_permutation(B)
    assert np.array_equal(xp.cpu().numpy(), x[cperm])
    assert spmv_error(A0, x, y2.cpu().numpy(), "f64") <= 1e-13
    ctx.release(B)
    ctx.release(A)


@pytest.mark.parametrize("k", [1, 5, 16])
def test_every_variant_is_bitwise_repeatable(ctx, k):
    """Each variant sums every row in a fixed order: two runs give the same bits."""
    A0 = synth.skewed_n4m(1, n=60_000)
    A = ctx.register(A0)
    B = ctx.permute(A, 4)
    X = torch_vec(synth.vector(A0.ncols, 2, k=k), torch.float64)
    for v in VARIANTS + [mx.variant(mx.VAR_SLAB, 12)]:
        if not _force(ctx, B, k, v):
            continue
        outs = []
        for _ in range(2):
            Y = torch.empty((A0.nrows, k) if k > 1 else (A0.nrows,), dtype=torch.float64,
                            device="cuda")
            ctx.spmv(B, X, Y)
            torch.cuda.synchronize()
            outs.append(Y.cpu().numpy().view(np.uint64).copy())
        assert np.array_equal(outs[0], outs[1]), hex(v)
    ctx.release(B)
    ctx.release(A)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", ["skewed", "wide", "clustered_n4096", "ragged"])
def test_window_equals_slab_bitwise(ctx, storage, name):
    """The window variant reads the same x values from LDS that the slab
    variant gathers, on the same layout: the same sums, bit for bit, in both
    the original (clustered) and the permuted matrix, for k classes 1 to 16."""
    A0 = dict(CSR_CASES)[name]()
    A = ctx.register(A0, storage)
    B = ctx.permute(A, 3)
    dt = torch.float64 if storage == "f64" else torch.float32
    for H in (A, B):
        for k in (1, 3, 8, 16):
            X = torch_vec(synth.vector(A0.ncols, 5, k=k), dt)
            outs = []
            for fam in (mx.VAR_SLAB, mx.VAR_WINDOW):
                for units in (16 | mx.SLAB_ONE_PER_CU, 4):
                    if not _force(ctx, H, k, mx.variant(fam, units)):
                        continue
                    Y = torch.full((A0.nrows, k) if k > 1 else (A0.nrows,), float("nan"),
                                   dtype=dt, device="cuda")
                    ctx.spmv(H, X, Y)
                    torch.cuda.synchronize()
                    outs.append(((fam, units), Y.cpu().numpy().copy()))
            by_units = {}
            for (fam, units), Y in outs:
                by_units.setdefault(units, []).append((fam, Y))
            for units, ys in by_units.items():
                if len(ys) == 2:
                    assert np.array_equal(ys[0][1].view(np.uint8), ys[1][1].view(np.uint8)), \
                        (name, storage, k, hex(units))
    ctx.release(B)
    ctx.release(A)


def test_runs_are_bitwise_deterministic(ctx):
    A0 = synth.skewed_n4m(1, n=40_000)
    A = ctx.register(A0)
    x = torch_vec(synth.vector(A0.ncols, 2), torch.float64)
    outs = []
    for _ in range(2):
        B = ctx.permute(A, 11)
        y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
        ctx.spmv(B, x, y)
        torch.cuda.synchronize()
        outs.append((ctx.export_csr(B), y.cpu().numpy(), ctx.entropy(B, 256, 256)))
        ctx.release(B)
    (c1, y1, h1), (c2, y2, h2) = outs
    for a, b in zip(c1, c2):
        assert np.array_equal(a, b)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    assert h1 == h2
    ctx.release(A)


# --- full-size configuration, as the benchmark runs it ------------------------------

def test_full_size_clustered_n2m(ctx):
    """n = 2,000,000 block-clustered matrix: permutation, permuted CSR,
    1024 x 1024 entropy and the tuned SpMV against the oracle in full."""
    A0 = synth.clustered_n2m(1)
    x = synth.vector(A0.ncols, 2)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    rperm, cperm = ctx.get_permutation(B)
    s_r, s_c = oracle.stream_seeds(3)
    assert np.array_equal(rperm, oracle.permutation(A0.nrows, s_r))
    assert np.array_equal(cperm, oracle.permutation(A0.ncols, s_c))
    er, ec, ev = expected_export(A0, rperm, cperm, "f64")
    gr, gc, gv = ctx.export_csr(B)
    assert np.array_equal(gr, er) and np.array_equal(gc, ec) and np.array_equal(gv, ev)
    bits, nats, hist = ctx.entropy(B, 1024, 1024, hist=True)
    ref = oracle.block_hist(A0.nrows, A0.ncols, er, ec, 1024, 1024)
    assert np.array_equal(hist, ref)
    assert (bits, nats) == oracle.entropy(ref)
    Bo = synth.CSR(A0.nrows, A0.ncols, er, ec, ev)
    xt = torch_vec(x, torch.float64)
    for H, Ho in ((A, A0), (B, Bo)):
        ctx.tune(H, 1)
        y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
        ctx.spmv(H, xt, y)
        torch.cuda.synchronize()
        assert spmv_error(Ho, x, y.cpu().numpy(), "f64") <= 1e-13
    # every slab layout the tuner picks for this workload on some box, forced
    for v in (mx.variant(mx.VAR_SLAB, 12), mx.variant(mx.VAR_SLAB, 16 | mx.SLAB_ONE_PER_CU),
              mx.variant(mx.VAR_SLAB, 20 | mx.SLAB_ONE_PER_CU),
              mx.variant(mx.VAR_SLAB, 24 | mx.SLAB_ONE_PER_CU)):
        ctx.set_variant(B, 1, v)
        y = torch.full((A0.nrows,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.spmv(B, xt, y)
        torch.cuda.synchronize()
        assert spmv_error(Bo, x, y.cpu().numpy(), "f64") <= 1e-13, hex(v)
    # and every window layout the tuner may pick for the original matrix
    for v in (mx.variant(mx.VAR_WINDOW, 16 | mx.SLAB_ONE_PER_CU),
              mx.variant(mx.VAR_WINDOW, 32 | mx.SLAB_ONE_PER_CU), mx.variant(mx.VAR_WINDOW, 32)):
        ctx.set_variant(A, 1, v)
        y = torch.full((A0.nrows,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.spmv(A, xt, y)
        torch.cuda.synchronize()
        assert spmv_error(A0, x, y.cpu().numpy(), "f64") <= 1e-13, hex(v)
    ctx.release(B)
    ctx.release(A)


# --- hierarchical entropy, gradient formats, fixed partition ------------------------

@pytest.mark.parametrize("case,grid", [("clustered_n4096", (64, 64)), ("skewed", (64, 64)),
                                       ("wide", (5, 1000)), ("ragged", (37, 23)),
                                       ("skewed", (1024, 1024))])    # several workgroups a region
def test_entropy_levels_exact(ctx, case, grid):
    A0 = dict(CSR_CASES)[case]()
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    levels = (1, 2, 4, 8)
    for H in (A, B):
        rp, col, _ = ctx.export_csr(H)
        ref_h = oracle.block_hist(A0.nrows, A0.ncols, rp, col, grid[0], grid[1])
        got = ctx.entropy_levels(H, grid[0], grid[1], levels)
        ref = oracle.entropy_levels(ref_h, levels)
        for (gb, gn), (rb, rn) in zip(got, ref):
            assert np.array_equal(gb, rb) and np.array_equal(gn, rn), case
        assert got[0][0][0, 0] == ctx.entropy(H, grid[0], grid[1])[0]
    ctx.release(B)
    ctx.release(A)


GRAD_CASES = CSR_CASES + [("one_row", lambda: synth.random_csr(1, 9, 0.5, 1)),
                          ("two_rows", lambda: synth.random_csr(2, 2, 1.0, 2)),
                          ("heavy", lambda: synth.heavy_clustered(30_000, 8, 0.02, 200, 2000.0, 4))]


@pytest.mark.parametrize("name,make", GRAD_CASES)
def test_gradient_formats_bit_exact(ctx, name, make):
    A0 = make()
    A = ctx.register(A0)
    for mode in (mx.ROWS | mx.GRADIENT, mx.ROWS | mx.COLS | mx.GRADIENT, mx.COLS | mx.GRADIENT):
        B = ctx.permute(A, 13, mode)
        rperm, cperm = ctx.get_permutation(B)
        er, ec, (rp, col, val) = oracle.permute_gradient(A0, 13, mode)
        assert np.array_equal(rperm, er), (name, mode)
        assert np.array_equal(cperm, ec), (name, mode)
        gr, gc, gv = ctx.export_csr(B)
        assert np.array_equal(gr, rp) and np.array_equal(gc, col) and np.array_equal(gv, val)
        ctx.release(B)
    ctx.release(A)


def test_fixed_partition_variant(ctx):
    A0 = synth.heavy_clustered(50_000, 8, 0.02, 256, 2000.0, 5)
    x = synth.vector(A0.ncols, 2, k=3)
    A = ctx.register(A0)
    B = ctx.permute(A, 3, mx.ROWS)
    rperm, cperm = ctx.get_permutation(B)
    Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
    for H, Ho in ((A, A0), (B, Bo)):
        for lanes in (1, 8, 64):
            ctx.set_variant(H, 3, mx.variant(mx.VAR_FIXED, lanes))
            Y = torch.full((A0.nrows, 3), float("nan"), dtype=torch.float64, device="cuda")
            ctx.spmv(H, torch_vec(x, torch.float64), Y)
            torch.cuda.synchronize()
            assert spmv_error(Ho, x, Y.cpu().numpy(), "f64") <= TOL["f64"], lanes
    ctx.release(B)
    ctx.release(A)


def test_coo_rows_across_many_tiles(ctx):
    """COO tiles cut rows: one row of 5000 entries (20 tiles), rows of 300,
    runs of empty rows at both ends and between."""
    rng = np.random.default_rng(17)
    lens = np.zeros(3000, np.int64)
    lens[5] = 5000
    lens[100:140] = 300
    lens[1000:2990:7] = rng.integers(1, 40, size=len(range(1000, 2990, 7)))
    rows = np.repeat(np.arange(3000), lens)
    cols = np.concatenate([rng.choice(6000, size=L, replace=False) for L in lens if L])
    A0 = synth.from_entries(3000, 6000, rows, cols, rng.uniform(-1, 1, len(rows)))
    A = ctx.register(A0)
    ctx.set_variant(A, 2, mx.variant(mx.VAR_COO))
    for k in (1, 2):
        X = synth.vector(A0.ncols, 5, k=k)
        Y = torch.full((A0.nrows, k) if k > 1 else (A0.nrows,), float("nan"),
                       dtype=torch.float64, device="cuda")
        ctx.set_variant(A, k, mx.variant(mx.VAR_COO))
        ctx.spmv(A, torch_vec(X, torch.float64), Y)
        torch.cuda.synchronize()
        assert spmv_error(A0, X, Y.cpu().numpy(), "f64") <= TOL["f64"], k
        ref = oracle.coo_spmm(A0.nrows, oracle.coo_rows(A0.row_ptr), A0.col, A0.val, X)
        assert np.array_equal(Y.cpu().numpy()[lens == 0], ref[lens == 0])    # exact zeros
    ctx.release(A)


def test_tuning_keeps_only_the_chosen_slab_layout(ctx):
    """The autotuner times several column-slab layouts; afterwards the matrix
    holds at most the one it chose (HBM accounting)."""
    A0 = synth.clustered_n2m(1, n=600_000)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    before = ctx.matrix_info(B).device_bytes
    v = ctx.tune(B, 1)
    delta = ctx.matrix_info(B).device_bytes - before
    layout = A0.nnz * 12                                  # uint32 word + FP64 value per entry
    if (v & 0xf00) in (mx.VAR_SLAB, mx.VAR_WINDOW):
        assert layout <= delta < layout + 4 * (1 << 22), (hex(v), delta)
    else:
        assert delta == 0, (hex(v), delta)
    x = torch_vec(synth.vector(A0.ncols, 2), torch.float64)
    y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
    ctx.spmv(B, x, y, flags=mx.SPACE_ORIGINAL)
    torch.cuda.synchronize()
    assert spmv_error(A0, synth.vector(A0.ncols, 2), y.cpu().numpy(), "f64") <= TOL["f64"]
    ctx.release(B)
    ctx.release(A)


def test_gather_probe(ctx):
    r_slab = ctx.probe_gather(8 * (12 << 16), 2_000_000, per_xcd=True)
    r_all = ctx.probe_gather(16 << 20, 2_000_000)
    assert 1e9 < r_slab < 1e13 and 1e9 < r_all < 1e13
    for bad in ((0, 10), (100, 10), (1 << 35, 10), (1024, 0)):
        with pytest.raises(mx.MxeError) as e:
            ctx.probe_gather(*bad)
        assert e.value.status == mx.ERR_INVALID_ARG


# --- other semirings: (min, +) and (or, and) ---------------------------------------

def _semiring_x(ncols, k, seed):
    X = synth.vector(ncols, seed, k=k)
    X[np.random.default_rng(seed).random(X.shape) < 0.3] = 0.0     # zeros matter for (or, and)
    return X


@pytest.mark.parametrize("name,make", CSR_CASES)
@pytest.mark.parametrize("k", [1, 3, 17])
def test_semiring_products_bit_exact(ctx, name, make, k):
    """FP64 storage: (min, +) and (or, and) equal the oracle bit for bit, in
    the permuted space and, through the permutations, in A's space."""
    A0 = make()
    X = _semiring_x(A0.ncols, k, 7)
    A = ctx.register(A0)
    B = ctx.permute(A, 3)
    rperm, cperm = ctx.get_permutation(B)
    Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
    shape = (A0.nrows, k) if k > 1 else (A0.nrows,)
    # the tuned kernel, then the column-slab kernel forced (64 KiB and 2 MiB slabs, and
    # 1 MiB slabs with row blocks for one workgroup per CU)
    for v in (None, mx.variant(mx.VAR_SLAB, 1), mx.variant(mx.VAR_SLAB, 32),
              mx.variant(mx.VAR_SLAB, 16 | mx.SLAB_ONE_PER_CU)):
        if v is not None and not (_force(ctx, A, k, v) and _force(ctx, B, k, v)):
            continue
        for sr in (mx.SR_MIN_PLUS, mx.SR_OR_AND):
            for H, Ho, flags, Xin in ((A, A0, 0, X), (B, Bo, 0, X[cperm]),
                                      (B, A0, mx.SPACE_ORIGINAL, X)):
                Y = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
                ctx.spmv_semiring(H, sr, torch_vec(Xin, torch.float64), Y, flags=flags)
                torch.cuda.synchronize()
                ref = oracle.spmm_semiring(sr, Ho.nrows, Ho.row_ptr, Ho.col, Ho.val, Xin)
                assert np.array_equal(Y.cpu().numpy(), ref.reshape(shape)), (name, sr, flags, v)
    ctx.release(B)
    ctx.release(A)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_semiring_products_reduced_storage(ctx, storage):
    A0 = synth.skewed_n4m(1, n=50_000)
    X = _semiring_x(A0.ncols, 4, 8)
    X32 = X.astype(np.float32).astype(np.float64)
    A = ctx.register(A0, storage)
    vals = oracle.stored_values(A0.val, storage)
    ctx.set_variant(A, 4, mx.variant(mx.VAR_SLAB, 4))             # the column-slab kernel
    for sr in (mx.SR_MIN_PLUS, mx.SR_OR_AND):
        Y = torch.full((A0.nrows, 4), float("nan"), dtype=torch.float32, device="cuda")
        ctx.spmv_semiring(A, sr, torch_vec(X, torch.float32), Y)
        torch.cuda.synchronize()
        got = Y.cpu().numpy().astype(np.float64)
        ref = oracle.spmm_semiring(sr, A0.nrows, A0.row_ptr, A0.col, vals, X32)
        if sr == mx.SR_OR_AND:
            assert np.array_equal(got, ref)
        else:                          # one FP32 rounding of each v + x, exact min
            assert np.array_equal(np.isinf(got), np.isinf(ref))
            fin = np.isfinite(ref)
            assert np.all(np.abs(got[fin] - ref[fin]) <= 2.0 ** -23 * (np.abs(ref[fin]) + 2.0))
    ctx.release(A)


def test_set_variant_validates(ctx):
    """Forced variants are checked before use: lane counts, families and slab
    sizes (with or without the one-workgroup-per-CU flag)."""
    A = ctx.register(synth.clustered_n4096(1))
    for bad in (mx.variant(mx.VAR_GROUP, 3), mx.variant(mx.VAR_GROUP, 128), 0x900,
                mx.variant(mx.VAR_SLAB, 0), mx.variant(mx.VAR_SLAB, 65),
                mx.variant(mx.VAR_SLAB, mx.SLAB_ONE_PER_CU),
                mx.variant(mx.VAR_SLAB, 65 | mx.SLAB_ONE_PER_CU), 0x1301, -1):
        with pytest.raises(mx.MxeError) as e:
            ctx.set_variant(A, 1, bad)
        assert e.value.status == mx.ERR_INVALID_ARG, hex(bad)
    for good in (mx.variant(mx.VAR_SLAB, 1), mx.variant(mx.VAR_SLAB, 1 | mx.SLAB_ONE_PER_CU),
                 mx.variant(mx.VAR_GROUP, 64)):
        ctx.set_variant(A, 1, good)
    ctx.release(A)


def test_semiring_rejects_unknown(ctx):
    A = ctx.register(synth.clustered_n4096(1))
    x = torch.zeros(4096, dtype=torch.float64, device="cuda")
    y = torch.zeros(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(mx.MxeError) as e:
        ctx.spmv_semiring(A, 7, x, y)
    assert e.value.status == mx.ERR_INVALID_ARG
    ctx.release(A)
