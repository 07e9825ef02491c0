"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times (autotuned variants, persistent batch plan, serving loop):
the skewed 4,000,000-row matrix in FP64 / FP32 / BF16 storage, the 64-matrix
batch and requests on full-size serving-pool matrices. Every output element
is compared with the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL, expected_export, spmv_error, torch_vec

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
mx = pytest.importorskip("paper_2308_00106_amd.mxe")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mx.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def skewed():
    return synth.skewed_n4m(1)


def test_skewed_full_size_permutation_csr_entropy(ctx, skewed):
    A0 = skewed
    print(f"skewed n={A0.nrows} nnz={A0.nnz}", flush=True)
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
    ctx.release(B)
    ctx.release(A)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_skewed_full_size_spmv(ctx, skewed, storage):
    """Tuned SpMV on the permuted matrix, in both index spaces, against the
    FP64 oracle on the original FP64 values."""
    A0 = skewed
    x = synth.vector(A0.ncols, 2)
    A = ctx.register(A0, storage)
    B = ctx.permute(A, 3)
    dt = torch.float64 if storage == "f64" else torch.float32
    xt = torch_vec(x, dt)
    v = ctx.tune(B, 1)
    y = torch.full((A0.nrows,), float("nan"), dtype=dt, device="cuda")
    ctx.spmv(B, xt, y, flags=mx.SPACE_ORIGINAL)
    torch.cuda.synchronize()
    err = spmv_error(A0, x, y.cpu().numpy().astype(np.float64), storage)
    assert err <= TOL[storage], (storage, hex(v), err)
    ctx.release(B)
    ctx.release(A)


def test_batch_full_size(ctx):
    """The 64-matrix batch (119M nonzeros, k in {1, 2, 4, 8, 16}, FP32) as one
    persistent launch replayed from a HIP graph, every output checked."""
    mats, ks = zip(*(synth.batch_member(i) for i in range(64)))
    print(f"batch nnz={sum(A.nnz for A in mats)}", flush=True)
    hs = [ctx.permute(ctx.register(A, "f32"), 1000 + i) for i, A in enumerate(mats)]
    Xs = [synth.vector(A.ncols, 50 + i, k=k) if k > 1 else synth.vector(A.ncols, 50 + i)
          for i, (A, k) in enumerate(zip(mats, ks))]
    Xt = [torch_vec(X, torch.float32) for X in Xs]
    Ys = [torch.full((A.nrows, k) if k > 1 else (A.nrows,), float("nan"), dtype=torch.float32,
                     device="cuda") for A, k in zip(mats, ks)]
    plan = ctx.batch_create(list(zip(hs, Xt, Ys)))
    for _ in range(2):
        ctx.batch_launch(plan)
    torch.cuda.synchronize()
    for i, (H, A0, X, Y) in enumerate(zip(hs, mats, Xs, Ys)):
        rperm, cperm = ctx.get_permutation(H)
        Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
        err = spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32")
        assert err <= TOL["f32"], (i, err)
    ctx.batch_destroy(plan)
    for H in hs:
        ctx.release(H)


def test_serving_full_size(ctx):
    """The serving loop on full-size pool matrices (block-clustered and skewed,
    up to 1.76M rows, FP32) in the benchmark's configuration (4 streams, 32 in
    flight, rounds of up to 8 items per launch, requests on one matrix merged
    up to k = 16): 48 requests of k = 1..8 submitted at once, every output
    checked against the FP64 oracle."""
    pool = [synth.serving_member(i) for i in (0, 1, 2, 3, 5)]
    print("serving pool rows", [A.nrows for A in pool], flush=True)
    hs = [ctx.permute(ctx.register(A, "f32"), 1000 + i) for i, A in enumerate(pool)]
    Bo = []
    for H, A0 in zip(hs, pool):
        rperm, cperm = ctx.get_permutation(H)
        Bo.append(synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm)))
    rng = np.random.default_rng(17)
    reqs = []
    for i in range(48):
        m = int(rng.integers(0, len(pool)))
        k = int(rng.integers(1, 9))
        X = synth.vector(pool[m].ncols, 300 + i, k=k) if k > 1 else synth.vector(pool[m].ncols, 300 + i)
        Y = torch.full((pool[m].nrows, k) if k > 1 else (pool[m].nrows,), float("nan"),
                       dtype=torch.float32, device="cuda")
        reqs.append((m, X, torch_vec(X, torch.float32), Y))
    ctx.serve_start(streams=2, max_inflight=32, max_batch=8, max_merge_k=8)
    tickets = [ctx.submit(hs[m], Xd, Y) for m, _, Xd, Y in reqs]
    for t in tickets:
        ctx.wait(t)
    ctx.serve_stop()
    for i, (m, X, _, Y) in enumerate(reqs):
        err = spmv_error(Bo[m], X, Y.cpu().numpy().astype(np.float64), "f32")
        assert err <= TOL["f32"], (i, m, err)
    for H in hs:
        ctx.release(H)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_slab_blocks_spread_over_whole_waves(ctx, storage):
    """Wide right-hand sides on a large matrix, where a row block's partial y
    no longer fits the LDS that two blocks per CU allow: the slab layout then
    spreads the rows over whole waves of the resident blocks. 700,000 rows,
    k = 8 and 16, the 2 MiB column-slab variants at one and two workgroups
    per CU forced, on the original and the permuted matrix, every output
    element against the oracle on the stored values."""
    A0 = synth.block_clustered(700_000, 8, 4096, 0.9, 21)
    print(f"wide-k n={A0.nrows} nnz={A0.nnz} {storage}", flush=True)
    A = ctx.register(A0, storage)
    B = ctx.permute(A, 4)
    rperm, cperm = ctx.get_permutation(B)
    Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
    dt = torch.float64 if storage == "f64" else torch.float32
    tol = TOL["f64"] if storage == "f64" else TOL["f32"]
    for H, Ho in ((A, A0), (B, Bo)):
        for k in (8, 16):
            X = synth.vector(A0.ncols, 30 + k, k=k)
            Xf = X if storage == "f64" else X.astype(np.float32).astype(np.float64)
            Xd = torch_vec(Xf, dt)
            for v in (mx.variant(mx.VAR_SLAB, 32), mx.variant(mx.VAR_SLAB, 32 | mx.SLAB_ONE_PER_CU)):
                ctx.set_variant(H, k, v)
                Y = torch.full((A0.nrows, k), float("nan"), dtype=dt, device="cuda")
                ctx.spmv(H, Xd, Y)
                torch.cuda.synchronize()
                err = spmv_error(Ho, Xf, Y.cpu().numpy().astype(np.float64), storage, ref_stored=True)
                assert err <= tol, (storage, k, hex(v), err)
    ctx.release(B)
    ctx.release(A)
