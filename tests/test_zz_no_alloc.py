"""GPU: the allocation-free batch entry point (mxe_spmv_batch_noalloc, for
callers that cannot allocate device memory) against the allocating one
(mxe_spmv_batch), through the C ABI: two calls in a row, the second with a
smaller input, each output bit for bit equal to the allocating call's and
within the FP tolerance of the FP64 oracle."""
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


def _members(n_mats, seed, rows):
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(n_mats):
        n = int(np.exp(rng.uniform(np.log(rows[0]), np.log(rows[1]))))
        if i % 2 == 0:
            mats.append(synth.block_clustered(n, rng.integers(8, 33, size=n), 4096, 0.9, seed + i))
        else:
            mats.append(synth.skewed_clustered(n, 2.0, 1.0, 256, 2000.0, seed + i))
    return mats


def _run_pair(ctx, mats, ks, storage, seed):
    """Prepares the items with mxe_spmv_batch (its output is the reference),
    then runs mxe_spmv_batch_noalloc into fresh outputs; returns both."""
    dt = torch.float64 if storage == "f64" else torch.float32
    hs = [ctx.permute(ctx.register(A, storage), seed) for A in mats]
    Xs = [synth.vector(A.ncols, seed + 10 + i, k=k) if k > 1 else synth.vector(A.ncols, seed + 10 + i)
          for i, (A, k) in enumerate(zip(mats, ks))]
    Xt = [torch_vec(X, dt) for X in Xs]

    def outs():
        return [torch.full((A.nrows, k) if k > 1 else (A.nrows,), float("nan"), dtype=dt,
                           device="cuda") for A, k in zip(mats, ks)]

    Y_ref, Y_new = outs(), outs()
    print(f"mxe_spmv_batch: {storage} rows {[A.nrows for A in mats]} k {ks}", flush=True)
    ctx.spmv_batch(list(zip(hs, Xt, Y_ref)))
    torch.cuda.synchronize()
    print("mxe_spmv_batch_noalloc: the same items", flush=True)
    ctx.spmv_batch_noalloc(list(zip(hs, Xt, Y_new)))
    torch.cuda.synchronize()
    return hs, Xs, Y_ref, Y_new


def _check(ctx, mats, ks, storage, hs, Xs, Y_ref, Y_new):
    for i, (A, k, H, X, Yr, Yn) in enumerate(zip(mats, ks, hs, Xs, Y_ref, Y_new)):
        assert torch.equal(Yr, Yn), f"item {i} (k={k}) differs from mxe_spmv_batch"
        rperm, cperm = ctx.get_permutation(H)
        Bo = synth.CSR(A.nrows, A.ncols, *oracle.permute_csr(A, rperm, cperm))
        err = spmv_error(Bo, X, Yn.cpu().numpy().astype(np.float64), storage)
        assert err <= TOL[storage], (i, k, err)


def test_noalloc_batch_matches_allocating_batch_twice(ctx):
    # first call: six FP32 matrices, k classes 1 ... 16
    mats1 = _members(6, 500, (10_000, 60_000))
    ks1 = [1, 2, 4, 8, 16, 3]
    r1 = _run_pair(ctx, mats1, ks1, "f32", 11)
    _check(ctx, mats1, ks1, "f32", *r1)
    # second call, right after, with a smaller input: two smaller FP64
    # matrices (fewer items, fewer work units, another value type; still
    # above one 4096-row diagonal block, so entries outside it exist)
    mats2 = _members(2, 600, (6_000, 9_000))
    ks2 = [1, 5]
    r2 = _run_pair(ctx, mats2, ks2, "f64", 12)
    _check(ctx, mats2, ks2, "f64", *r2)
    for h in r1[0] + r2[0]:
        ctx.release(h)


def test_noalloc_batch_refuses_what_it_cannot_do(ctx):
    A = _members(1, 700, (6_000, 7_000))[0]
    H = ctx.permute(ctx.register(A, "f32"), 13)
    X = torch_vec(synth.vector(A.ncols, 14), torch.float32)
    Y = torch.empty(A.nrows, dtype=torch.float32, device="cuda")
    # not tuned yet for k = 1: nothing is tuned or built here
    with pytest.raises(mx.MxeError) as e:
        ctx.spmv_batch_noalloc([(H, X, Y)])
    assert e.value.status == mx.ERR_UNSUPPORTED
    print("mxe_spmv_batch: prepares one item", flush=True)
    ctx.spmv_batch([(H, X, Y)])
    with pytest.raises(mx.MxeError) as e:
        ctx.spmv_batch_noalloc([(H, X, Y)] * (mx.NOALLOC_MAX_ITEMS + 1))
    assert e.value.status == mx.ERR_INVALID_ARG
    print("mxe_spmv_batch_noalloc: one prepared item", flush=True)
    ctx.spmv_batch_noalloc([(H, X, Y)])
    torch.cuda.synchronize()
    ctx.release(H)
