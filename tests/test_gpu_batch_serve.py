"""GPU: uneven multi-matrix batches in one persistent launch (plain and
replayed from a HIP graph), and the continuous-batching serving loop. Each
result is checked against the FP64 oracle and against the same product run
alone."""
import threading

import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL, spmv_error, torch_vec

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


def _pool(n_mats, seed, rows=(10_000, 60_000)):
    """Small stand-ins for the batch and serving pools: log-uniform sizes,
    block-clustered (8-32 per row) and skewed clustered structures."""
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(n_mats):
        n = int(np.exp(rng.uniform(np.log(rows[0]), np.log(rows[1]))))
        if i % 2 == 0:
            mats.append(synth.block_clustered(n, rng.integers(8, 33, size=n), 4096, 0.9, seed + i))
        else:
            mats.append(synth.skewed_clustered(n, 2.0, 1.0, 256, 2000.0, seed + i))
    return mats


def _rand_x(A, k, seed):
    return synth.vector(A.ncols, seed, k=k) if k > 1 else synth.vector(A.ncols, seed)


def _empty_y(A, k):
    return torch.full((A.nrows, k) if k > 1 else (A.nrows,), float("nan"), dtype=torch.float32,
                      device="cuda")


# --- batches ---------------------------------------------------------------------

def test_batch_uneven_multi_rhs(ctx):
    mats = _pool(8, 100)
    ks = [1, 2, 4, 8, 16, 3, 5, 16]
    handles = [ctx.permute(ctx.register(A, "f32"), 7) for A in mats]
    B0 = []
    for H, A in zip(handles, mats):
        rperm, cperm = ctx.get_permutation(H)
        B0.append(synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm)))
    Xs = [_rand_x(A, k, 10 + i) for i, (A, k) in enumerate(zip(mats, ks))]
    Xt = [torch_vec(X, torch.float32) for X in Xs]
    Ys = [_empty_y(A, k) for A, k in zip(mats, ks)]
    ctx.spmv_batch(list(zip(handles, Xt, Ys)))
    torch.cuda.synchronize()
    for Bo, X, Y, k in zip(B0, Xs, Ys, ks):
        assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"], k
    # same products one at a time
    for H, Bo, X, Xd, Y, k in zip(handles, B0, Xs, Xt, Ys, ks):
        Ya = torch.empty_like(Y)
        ctx.spmv(H, Xd, Ya)
        torch.cuda.synchronize()
        d = np.abs(Ya.cpu().numpy().astype(np.float64) - Y.cpu().numpy().astype(np.float64))
        den = oracle.spmm(Bo.nrows, Bo.row_ptr, Bo.col, np.abs(Bo.val), np.abs(X))
        den = den.reshape(d.shape)
        assert np.all(d <= TOL["f32"] * np.where(den == 0, 1, den)), k


def test_batch_plan_graph_replays(ctx):
    """The plan's graph replays correctly several times, with eager work and
    synchronisation between replays, with new X / Y buffers, and after its
    matrices' handles are released (the plan keeps them alive)."""
    mats = _pool(5, 200)
    ks = [1, 4, 16, 2, 8]
    handles = [ctx.permute(ctx.register(A, "f32"), 9) for A in mats]
    B0 = []
    for H, A in zip(handles, mats):
        rperm, cperm = ctx.get_permutation(H)
        B0.append(synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm)))
    Xs = [_rand_x(A, k, 20 + i) for i, (A, k) in enumerate(zip(mats, ks))]
    Xt = [torch_vec(X, torch.float32) for X in Xs]
    Ys = [_empty_y(A, k) for A, k in zip(mats, ks)]
    plan = ctx.batch_create(list(zip(handles, Xt, Ys)))
    for replay in range(3):
        for Y in Ys:
            Y.fill_(float("nan"))
        ctx.batch_launch(plan)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()        # eager work between replays
        for Bo, X, Y in zip(B0, Xs, Ys):
            assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"], replay
    # new vectors: the descriptors are rewritten before the replay
    Xs2 = [_rand_x(A, k, 30 + i) for i, (A, k) in enumerate(zip(mats, ks))]
    Xt2 = [torch_vec(X, torch.float32) for X in Xs2]
    Ys2 = [_empty_y(A, k) for A, k in zip(mats, ks)]
    for _ in range(2):
        ctx.batch_launch(plan, list(zip(handles, Xt2, Ys2)))
        torch.cuda.synchronize()
        for Bo, X, Y in zip(B0, Xs2, Ys2):
            assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"]
    with pytest.raises(mx.MxeError):
        ctx.batch_launch(plan, list(zip(handles[::-1], Xt2[::-1], Ys2[::-1])))
    # the plan keeps its matrices alive: released handles still replay, with
    # the planned vectors and with new ones
    for H in handles:
        ctx.release(H)
    for Y in Ys2:
        Y.fill_(float("nan"))
    ctx.batch_launch(plan)
    torch.cuda.synchronize()
    for Bo, X, Y in zip(B0, Xs2, Ys2):
        assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"]
    ctx.batch_destroy(plan)


def _slab_units(A, k, storage):
    """Slab size (in 64 KiB units) that cuts x into about 8 slabs."""
    xb = 8 if storage == "f64" else 4
    kc = 1 << (k - 1).bit_length()
    return max(1, -(-(A.ncols * xb * kc) // (8 * 65536)))


def test_batch_slab_units(ctx):
    """Items whose variant is the column-slab kernel run as the blocks of its
    layout inside the persistent launch, next to row-tile items: k equal to its
    class (whole-row vector loads) and below it, a padded X (ldx > k, no vector
    loads), FP64 / FP32 / BF16 storage. Checked against the oracle directly and
    after graph replays, which agree bit for bit with each other."""
    mats = _pool(7, 500, rows=(30_000, 90_000))
    storages = ["f32", "f32", "f64", "bf16", "f32", "f64", "f32"]
    ks = [1, 4, 3, 16, 8, 2, 4]
    slab = [True, True, True, True, False, True, True]
    padded = [False, False, False, False, False, False, True]
    handles = [ctx.permute(ctx.register(A, st), 13) for A, st in zip(mats, storages)]
    B0 = []
    for H, A, k, st, sl in zip(handles, mats, ks, storages, slab):
        rperm, cperm = ctx.get_permutation(H)
        B0.append(synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm)))
        var = mx.variant(mx.VAR_SLAB, _slab_units(A, k, st)) if sl else mx.variant(mx.VAR_GROUP, 8)
        ctx.set_variant(H, k, var)
    Xs = [_rand_x(A, k, 70 + i) for i, (A, k) in enumerate(zip(mats, ks))]
    dts = [torch.float64 if st == "f64" else torch.float32 for st in storages]
    Xt = []
    for X, dt, pad, k in zip(Xs, dts, padded, ks):
        if pad:                                   # ldx = k + 1: rows off the 16-byte grid
            buf = torch.zeros((X.shape[0], k + 1), dtype=dt, device="cuda")
            buf[:, :k] = torch_vec(X, dt)
            Xt.append(buf[:, :k])
        else:
            Xt.append(torch_vec(X, dt))
    Ys = [torch.full((A.nrows, k) if k > 1 else (A.nrows,), float("nan"), dtype=dt, device="cuda")
          for A, k, dt in zip(mats, ks, dts)]
    print("slab batch", [(A.nrows, k, st) for A, k, st in zip(mats, ks, storages)], flush=True)
    ctx.spmv_batch(list(zip(handles, Xt, Ys)))
    torch.cuda.synchronize()
    for i, (Bo, X, Y, st) in enumerate(zip(B0, Xs, Ys, storages)):
        assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), st) <= TOL[st], (i, st)
    first = [Y.clone() for Y in Ys]
    plan = ctx.batch_create(list(zip(handles, Xt, Ys)))
    for replay in range(3):
        for Y in Ys:
            Y.fill_(float("nan"))
        ctx.batch_launch(plan)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()        # eager work between replays
        for i, (Y, Y1) in enumerate(zip(Ys, first)):
            assert torch.equal(Y, Y1), (replay, i)
    ctx.batch_destroy(plan)
    for H in handles:
        ctx.release(H)


def test_batch_slab_layout_within_budget():
    """A batch gives a slab-tuned item that stays on one XCD (here eight equal
    items, none above an eighth of the batch) a second layout with row blocks
    sized for one XCD; when the HBM budget has no room for it the items run on
    their tuned layout, with a correct result either way. An item alone in a
    batch is spread over every XCD and runs on its tuned layout."""
    A0 = synth.clustered_n2m(1, n=200_000)
    k = 4
    X = synth.vector(A0.ncols, 6, k=k)

    def setup(c):
        A = c.register(A0, "f32")
        H = c.permute(A, 5)
        c.set_variant(H, k, mx.variant(mx.VAR_SLAB, 4))
        Xd = torch_vec(X, torch.float32)
        Y = torch.empty((A0.nrows, k), dtype=torch.float32, device="cuda")
        c.spmv(H, Xd, Y)                                  # builds the tuned layout
        torch.cuda.synchronize()
        rperm, cperm = c.get_permutation(H)
        Bo = synth.CSR(A0.nrows, A0.ncols, *oracle.permute_csr(A0, rperm, cperm))
        return A, H, Xd, Bo

    def run_batch(c, H, Xd, Bo, n=8):
        Ys = [torch.full((A0.nrows, k), float("nan"), dtype=torch.float32, device="cuda")
              for _ in range(n)]
        c.spmv_batch([(H, Xd, Y) for Y in Ys])
        torch.cuda.synchronize()
        for Y in Ys:
            assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"]

    with mx.Context(0) as c1:
        A, H, Xd, Bo = setup(c1)
        resident = c1.matrix_info(A).device_bytes + c1.matrix_info(H).device_bytes
        before = c1.matrix_info(H).device_bytes
        run_batch(c1, H, Xd, Bo, n=1)
        assert c1.matrix_info(H).device_bytes == before   # spread: the tuned layout ran
        run_batch(c1, H, Xd, Bo)
        grown = c1.matrix_info(H).device_bytes - before
        assert grown >= A0.nnz * 8                        # the per-XCD layout was built
    with mx.Context(0, budget_bytes=resident + grown // 2) as c2:
        A, H, Xd, Bo = setup(c2)
        before = c2.matrix_info(H).device_bytes
        run_batch(c2, H, Xd, Bo)
        assert c2.matrix_info(H).device_bytes == before   # no room: the tuned layout ran


def test_batch_mixed_storage(ctx):
    """FP64, FP32 and BF16 items in one persistent launch (the instance that
    carries every value type), directly and from a graph replay."""
    mats = _pool(6, 400)
    storages = ["f64", "f32", "bf16", "f64", "bf16", "f32"]
    ks = [1, 4, 2, 16, 3, 8]
    handles = [ctx.permute(ctx.register(A, st), 11) for A, st in zip(mats, storages)]
    B0 = []
    for H, A in zip(handles, mats):
        rperm, cperm = ctx.get_permutation(H)
        B0.append(synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm)))
    Xs = [_rand_x(A, k, 60 + i) for i, (A, k) in enumerate(zip(mats, ks))]
    dts = [torch.float64 if st == "f64" else torch.float32 for st in storages]
    Xt = [torch_vec(X, dt) for X, dt in zip(Xs, dts)]
    Ys = [torch.full((A.nrows, k) if k > 1 else (A.nrows,), float("nan"), dtype=dt, device="cuda")
          for A, k, dt in zip(mats, ks, dts)]
    ctx.spmv_batch(list(zip(handles, Xt, Ys)))
    torch.cuda.synchronize()
    for Bo, X, Y, st in zip(B0, Xs, Ys, storages):
        assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), st) <= TOL[st], st
    plan = ctx.batch_create(list(zip(handles, Xt, Ys)))
    for Y in Ys:
        Y.fill_(float("nan"))
    ctx.batch_launch(plan)
    torch.cuda.synchronize()
    for Bo, X, Y, st in zip(B0, Xs, Ys, storages):
        assert spmv_error(Bo, X, Y.cpu().numpy().astype(np.float64), st) <= TOL[st], st
    ctx.batch_destroy(plan)
    for H in handles:
        ctx.release(H)


# --- serving ---------------------------------------------------------------------------

def _alone_denominator(ref_csr, X, shape):
    den = oracle.spmm(ref_csr.nrows, ref_csr.row_ptr, ref_csr.col, np.abs(ref_csr.val), np.abs(X))
    return den.reshape(shape)


def _serving_run(ctx, mats, handles, variants, max_batch, seed, max_merge_k=1, storage="f32"):
    """64 requests from two submitter threads on a few matrices (so requests
    on one matrix overlap on several streams), mixed k and index spaces; each
    result is compared with the same product run alone afterwards: bit for
    bit when every request runs as its own product (max_batch and max_merge_k
    1: the same kernel on the same data), else within the tolerance element
    by element (a batch runs an item on its own layout and work units, a
    merged item sums its columns in another order), and against the oracle
    either way."""
    dt = torch.float64 if storage == "f64" else torch.float32
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(64):
        m = int(rng.integers(0, len(mats)))
        k = int(rng.integers(1, 9))
        flags = mx.SPACE_ORIGINAL if r % 3 == 0 else mx.SPACE_PERMUTED
        X = _rand_x(mats[m], k, seed * 1000 + r)
        Y = torch.full((mats[m].nrows, k) if k > 1 else (mats[m].nrows,), float("nan"), dtype=dt,
                       device="cuda")
        reqs.append((m, k, flags, X, torch_vec(X, dt), Y))
    for m, per_k in variants.items():
        for k, var in per_k.items():
            ctx.set_variant(handles[m], k, var)
    ctx.serve_start(streams=4, max_inflight=16, max_batch=max_batch, max_merge_k=max_merge_k)
    tickets = [None] * len(reqs)

    def submitter(lo, hi):
        for i in range(lo, hi):
            m, k, flags, _, Xd, Y = reqs[i]
            tickets[i] = ctx.submit(handles[m], Xd, Y, flags)

    th = [threading.Thread(target=submitter, args=(i * 32, (i + 1) * 32)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    lat = [ctx.wait(t) for t in tickets]
    ctx.serve_stop()
    assert all(v > 0 for v in lat)
    perms = {m: ctx.get_permutation(h) for m, h in enumerate(handles)}
    for i, (m, k, flags, X, Xd, Y) in enumerate(reqs):
        Ya = torch.full_like(Y, float("nan"))
        ctx.spmv(handles[m], Xd, Ya, flags=flags)
        torch.cuda.synchronize()
        A = mats[m]
        if flags == mx.SPACE_ORIGINAL:
            ref_csr = A
        else:
            rperm, cperm = perms[m]
            ref_csr = synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm))
        y_mix = Y.cpu().numpy().astype(np.float64)
        y_alone = Ya.cpu().numpy().astype(np.float64)
        if max_batch == 1 and max_merge_k == 1:
            assert np.array_equal(y_mix.view(np.uint64), y_alone.view(np.uint64)), (i, m, k, flags)
        else:
            den = _alone_denominator(ref_csr, X, y_mix.shape)
            d = np.abs(y_mix - y_alone)
            assert np.all(d <= TOL[storage] * np.where(den == 0, 1, den)), (i, m, k, flags)
        assert spmv_error(ref_csr, X, y_mix, storage) <= TOL[storage], (i, m, k, flags)
    for m, per_k in variants.items():
        for k in per_k:
            ctx.set_variant(handles[m], k, 0)


def test_serving_mix_matches_alone(ctx):
    """Concurrent requests on the same matrices, with the merge-path and COO
    kernels forced on two of them (their carries are per launch), agree with
    the products run alone: bitwise when each request is its own product,
    within tolerance when rounds run as persistent batch launches."""
    mats = _pool(4, 300, rows=(20_000, 80_000))
    handles = [ctx.permute(ctx.register(A, "f32"), 5) for A in mats]
    merge = mx.variant(mx.VAR_MERGE)
    coo = mx.variant(mx.VAR_COO)
    variants = {0: {1: merge, 2: merge, 4: merge, 8: coo, 16: coo},
                1: {1: coo, 2: coo, 4: coo, 8: coo, 16: coo}}
    _serving_run(ctx, mats, handles, variants, max_batch=1, seed=1)
    _serving_run(ctx, mats, handles, variants, max_batch=8, seed=2)
    _serving_run(ctx, mats, handles, variants, max_batch=8, seed=3, max_merge_k=16)
    _serving_run(ctx, mats, handles, {}, max_batch=8, seed=4, max_merge_k=16)
    _serving_run(ctx, mats, handles, {}, max_batch=64, seed=5, max_merge_k=7)
    _serving_run(ctx, mats, handles, {}, max_batch=1, seed=6, max_merge_k=16)
    for H in handles:
        ctx.release(H)
    # FP64 storage: merged right-hand sides packed as 8-byte values
    handles = [ctx.permute(ctx.register(A, "f64"), 5) for A in mats]
    _serving_run(ctx, mats, handles, {}, max_batch=8, seed=7, max_merge_k=16, storage="f64")
    for H in handles:
        ctx.release(H)


@pytest.mark.parametrize("family", ["merge", "coo"])
def test_carry_variants_on_two_streams(ctx, family):
    """Products of one matrix issued alternately on two streams (so launches
    may overlap) equal the same products issued one by one, bit for bit."""
    A0 = synth.skewed_clustered(150_000, 2.0, 1.0, 256, 2000.0, 31)
    A = ctx.register(A0, "f32")
    H = ctx.permute(A, 3)
    var = mx.variant(mx.VAR_MERGE if family == "merge" else mx.VAR_COO)
    ctx.set_variant(H, 1, var)
    Xs = [torch_vec(synth.vector(A0.ncols, 40 + i), torch.float32) for i in range(12)]
    ref = []
    for X in Xs:
        Y = torch.empty(A0.nrows, dtype=torch.float32, device="cuda")
        ctx.spmv(H, X, Y)
        torch.cuda.synchronize()
        ref.append(Y)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for i, X in enumerate(Xs):
        Y = torch.full((A0.nrows,), float("nan"), dtype=torch.float32, device="cuda")
        ctx.spmv(H, X, Y, stream=streams[i % 2])
        outs.append(Y)
    torch.cuda.synchronize()
    for i, (Y, R) in enumerate(zip(outs, ref)):
        assert torch.equal(Y, R), i
    ctx.release(H)
    ctx.release(A)


def test_release_waits_for_queued_products(ctx):
    """A matrix released while products on it are still queued on a side
    stream keeps its memory until they have ended: they read intact memory,
    and a matrix registered, permuted and multiplied right after on the
    default stream (its memory may come from the freed blocks) is exact."""
    A0 = synth.clustered_n2m(3, n=400_000)
    A = ctx.register(A0, "f64")
    B = ctx.permute(A, 11)
    X = torch_vec(np.random.default_rng(2).uniform(-1, 1, A0.ncols), torch.float64)
    ref = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
    ctx.spmv(B, X, ref)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    outs = [torch.full((A0.nrows,), float("nan"), dtype=torch.float64, device="cuda")
            for _ in range(12)]
    torch.cuda.synchronize()
    for Y in outs:
        ctx.spmv(B, X, Y, stream=side)
    ctx.release(B)
    ctx.release(A)
    A1 = synth.clustered_n2m(4, n=400_000)
    C = ctx.register(A1, "f64")
    D = ctx.permute(C, 12)
    Z = torch.empty(A1.nrows, dtype=torch.float64, device="cuda")
    ctx.spmv(D, X, Z)
    torch.cuda.synchronize()
    for i, Y in enumerate(outs):
        assert torch.equal(Y, ref), i
    rperm, cperm = ctx.get_permutation(D)
    Dp = synth.CSR(A1.nrows, A1.ncols, *oracle.permute_csr(A1, rperm, cperm))
    err = spmv_error(Dp, X.cpu().numpy(), Z.cpu().numpy(), "f64")
    assert err <= TOL["f64"], err
    ctx.release(D)
    ctx.release(C)


def test_serving_budget_admission_and_busy_release(ctx):
    A0 = synth.clustered_n2m(1, n=200_000)
    with mx.Context(0, budget_bytes=0) as probe:
        H = probe.register(A0, "f32")
        resident = probe.matrix_info(H).device_bytes
    vec = 8 * (A0.nrows + A0.ncols) * 4            # one request of k = 8 in FP32
    # room for the matrix and one in-flight request: requests run one at a time
    with mx.Context(0, budget_bytes=resident + vec + 1024) as c2:
        H = c2.register(A0, "f32")
        c2.serve_start(streams=2, max_inflight=8, max_batch=1, max_merge_k=1)
        X = synth.vector(A0.ncols, 3, k=8)
        Xd = torch_vec(X, torch.float32)
        Ys = [torch.empty((A0.nrows, 8), dtype=torch.float32, device="cuda") for _ in range(6)]
        ts = [c2.submit(H, Xd, Y) for Y in Ys]
        with pytest.raises(mx.MxeError) as e:
            c2.release(H)
        assert e.value.status == mx.ERR_BUSY
        for t in ts:
            c2.wait(t)
        for Y in Ys:
            assert spmv_error(A0, X, Y.cpu().numpy().astype(np.float64), "f32") <= TOL["f32"]
        # a request that can never fit the budget fails instead of waiting
        X16 = torch_vec(synth.vector(A0.ncols, 4, k=16), torch.float32)
        Y16 = torch.empty((A0.nrows, 16), dtype=torch.float32, device="cuda")
        t = c2.submit(H, X16, Y16)
        with pytest.raises(mx.MxeError) as e:
            c2.wait(t)
        assert e.value.status == mx.ERR_BUDGET
        c2.serve_stop()
        c2.release(H)


def test_wait_timeout_and_unknown_ticket(ctx):
    A0 = synth.clustered_n2m(1, n=100_000)
    H = ctx.register(A0, "f32")
    ctx.serve_start(streams=1, max_inflight=1, max_batch=1, max_merge_k=1)
    X = torch_vec(synth.vector(A0.ncols, 3), torch.float32)
    Y = torch.empty(A0.nrows, dtype=torch.float32, device="cuda")
    t = ctx.submit(H, X, Y)
    ctx.wait(t)
    with pytest.raises(mx.MxeError) as e:
        ctx.wait(t)                      # retired
    assert e.value.status == mx.ERR_NOT_FOUND
    ctx.serve_stop()
    with pytest.raises(mx.MxeError):
        ctx.submit(H, X, Y)              # loop stopped
    ctx.release(H)
