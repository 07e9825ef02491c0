"""Extra measurements for bench.py --extras (one GPU):

  skewed      4,000,000-row CSR, lognormal row lengths capped at 256, columns
              Gaussian around the diagonal; values stored FP64 / FP32 / BF16
              (FP32 accumulation for the reduced ones): permuted vs original
              SpMV and the error against the FP64 oracle on the FP64 values.
  batch       64 matrices (rows log-uniform in [10k, 500k], 8-32 nnz per row,
              block-clustered), k in {1, 2, 4, 8, 16}, FP32; one persistent
              launch replayed from a HIP graph.
  heavy       2,000,000-row CSR, 8 nnz per row except one contiguous band of
              1% of the rows with 512 each (heavy clustered rows): SpMV with
              the fixed equal-row partition (no counting), the COO kernel and
              the tuned count-aware variant on the original, R, RC and
              gradient (G-R, G-RC) orderings, plus the hierarchical 2D
              entropy of each.
  semiring    the n = 2,000,000 block-clustered matrix (FP64): (min, +) and
              (or, and) products, original vs permuted, against the (+, *) one.
  serving     32 resident permuted matrices of 50k-2M rows (FP32), requests of
              1-8 right-hand sides on a random matrix; closed-loop saturation
              rate, then open-loop Poisson arrivals at 0.5 and 0.8 of it:
              p50 / p99 latency and aggregate GB/s.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import synth


def _bytes(A, val_bytes, vec_bytes, k):
    return A.nnz * (val_bytes + 4) + (A.nrows + 1) * 4 + k * (A.ncols + A.nrows) * vec_bytes


def _generate(fn, count, workers=8):
    """fn(0), ..., fn(count - 1) on a thread pool (each is a pure function of
    its index; numpy releases the GIL in the heavy parts)."""
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, range(count)))


def _time(ctx, m, X, Y, reps, stream, flags=0):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.spmv(m, X, Y, flags=flags, stream=stream)
    e0.record(stream)
    for _ in range(reps):
        ctx.spmv(m, X, Y, flags=flags, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def skewed(ctx, log, n=4_000_000, reps=50):
    import torch
    from paper_2308_00106_amd import mxe as mx
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    A0 = synth.skewed_n4m(1, n=n)
    x = synth.vector(A0.ncols, 2)
    log(f"skewed: generated n={n} nnz={A0.nnz} in {time.perf_counter() - t:.1f}s")
    yref = oracle.spmv(A0, x)
    out = {"n": n, "nnz": A0.nnz, "max_row": int(A0.row_lengths().max())}
    for st in ("f64", "f32", "bf16"):
        A = ctx.register(A0, st)
        B = ctx.permute(A, 3, stream=stream)
        tdt = torch.float64 if st == "f64" else torch.float32
        xt = torch.from_numpy(x).to(device="cuda", dtype=tdt)
        y = torch.empty(A0.nrows, dtype=tdt, device="cuda")
        r = {}
        for name, H in (("permuted", B), ("original", A)):
            v = ctx.tune(H, 1, stream=stream)
            us = _time(ctx, H, xt, y, reps, stream)
            vb = {"f64": 8, "f32": 4, "bf16": 2}[st]
            nb = _bytes(A0, vb, 8 if st == "f64" else 4, 1)
            r[name] = {"us": round(us, 2), "gbs": round(nb / (us * 1e-6) / 1e9, 1), "variant": hex(v)}
        r["permuted_over_original"] = round(r["original"]["us"] / r["permuted"]["us"], 4)
        ctx.spmv(B, xt, y, flags=mx.SPACE_ORIGINAL, stream=stream)
        torch.cuda.synchronize()
        r["max_normalized_error_vs_fp64_oracle"] = oracle.normalized_error(
            A0.nrows, A0.row_ptr, A0.col, A0.val, x, y.cpu().numpy().astype(np.float64), yref)
        r["entropy_bits_1024"] = {"original": ctx.entropy(A, 1024, 1024)[0],
                                  "permuted": ctx.entropy(B, 1024, 1024)[0]}
        out[st] = r
        log(f"skewed {st}: {r}")
        ctx.release(B)
        ctx.release(A)
    return out


def heavy(ctx, log, n=2_000_000, reps=50):
    import torch
    from paper_2308_00106_amd import mxe as mx
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    A0 = synth.heavy_clustered(n, 8, 0.01, 512, 2000.0, 7)
    x = synth.vector(A0.ncols, 2)
    log(f"heavy: generated n={n} nnz={A0.nnz} in {time.perf_counter() - t:.1f}s")
    yref = oracle.spmv(A0, x)
    nb = _bytes(A0, 8, 8, 1)
    out = {"n": n, "nnz": A0.nnz, "heavy_rows": int((A0.row_lengths() == 512).sum())}
    A = ctx.register(A0)
    xt = torch.from_numpy(x).to(device="cuda")
    y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
    forms = {"original": None, "R": mx.ROWS, "RC": mx.ROWS | mx.COLS,
             "G-R": mx.ROWS | mx.GRADIENT, "G-RC": mx.ROWS | mx.COLS | mx.GRADIENT}
    for name, mode in forms.items():
        H = A if mode is None else ctx.permute(A, 3, mode, stream=stream)
        r = {}
        for lanes in (8, 32):
            ctx.set_variant(H, 1, mx.variant(mx.VAR_FIXED, lanes))
            us = _time(ctx, H, xt, y, reps, stream)
            r[f"fixed_l{lanes}_us"] = round(us, 2)
        ctx.set_variant(H, 1, mx.variant(mx.VAR_COO))     # 16 B per entry: row, column, value
        r["coo_us"] = round(_time(ctx, H, xt, y, reps, stream), 2)
        v = ctx.tune(H, 1, stream=stream)
        us = _time(ctx, H, xt, y, reps, stream)
        r["tuned_us"] = round(us, 2)
        r["tuned_variant"] = hex(v)
        r["tuned_gbs"] = round(nb / (us * 1e-6) / 1e9, 1)
        ctx.spmv(H, xt, y, flags=mx.SPACE_ORIGINAL, stream=stream)
        torch.cuda.synchronize()
        r["max_normalized_error_vs_fp64_oracle"] = oracle.normalized_error(
            A0.nrows, A0.row_ptr, A0.col, A0.val, x, y.cpu().numpy(), yref)
        r["entropy_bits_64"] = ctx.entropy(H, 64, 64)[0]
        t0 = time.perf_counter()
        lv = ctx.entropy_levels(H, 64, 64, (2, 4, 8), stream=stream)
        r["levels_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        r["levels_bits"] = {L: np.round(b, 3).tolist() for L, (b, _) in zip((2, 4), lv[:2])}
        r["levels8_bits_min_max"] = [round(float(lv[2][0].min()), 3), round(float(lv[2][0].max()), 3)]
        out[name] = r
        log(f"heavy {name}: {r}")
        if mode is not None:
            ctx.release(H)
    ctx.release(A)
    return out


def semiring(ctx, log, n=2_000_000, reps=50):
    import torch
    from paper_2308_00106_amd import mxe as mx
    stream = torch.cuda.current_stream()
    A0 = synth.clustered_n2m(1, n=n)
    A = ctx.register(A0)
    B = ctx.permute(A, 3, stream=stream)
    nb = _bytes(A0, 8, 8, 1)
    out = {"n": n, "nnz": A0.nnz}
    for name, H in (("original", A), ("permuted", B)):
        x = torch.from_numpy(synth.vector(A0.ncols, 2)).to(device="cuda")
        y = torch.empty(A0.nrows, dtype=torch.float64, device="cuda")
        r = {}
        for sr_name, sr in (("min_plus", mx.SR_MIN_PLUS), ("or_and", mx.SR_OR_AND)):
            ctx.spmv_semiring(H, sr, x, y, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                ctx.spmv_semiring(H, sr, x, y, stream=stream)
            e1.record(stream)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            r[sr_name] = {"us": round(us, 2), "gbs": round(nb / (us * 1e-6) / 1e9, 1)}
        ctx.tune(H, 1, stream=stream)
        r["plus_times_tuned_us"] = round(_time(ctx, H, x, y, reps, stream), 2)
        out[name] = r
        log(f"semiring {name}: {r}")
    ctx.release(B)
    ctx.release(A)
    return out


def batch(ctx, log, count=64, replays=20):
    import torch
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    members = _generate(synth.batch_member, count)
    mats = [A for A, _ in members]
    ks = [k for _, k in members]
    log(f"batch: generated {count} matrices, {sum(A.nnz for A in mats)} nnz in "
        f"{time.perf_counter() - t:.1f}s")
    hs = [ctx.permute(ctx.register(A, "f32"), 1000 + i, stream=stream) for i, A in enumerate(mats)]
    Xs = [torch.rand((A.ncols, k), dtype=torch.float32, device="cuda") * 2 - 1 for A, k in zip(mats, ks)]
    Ys = [torch.empty((A.nrows, k), dtype=torch.float32, device="cuda") for A, k in zip(mats, ks)]
    items = list(zip(hs, Xs, Ys))
    plan = ctx.batch_create(items)
    ctx.batch_launch(plan, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(replays):
        ctx.batch_launch(plan, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / replays
    # reference: the same products one launch per item, each with its own tuned variant
    for h, X, Y in items:
        ctx.spmv(h, X, Y, stream=stream)
    e0.record(stream)
    for _ in range(5):
        for h, X, Y in items:
            ctx.spmv(h, X, Y, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us_items = e0.elapsed_time(e1) * 1e3 / 5
    nb = sum(_bytes(A, 4, 4, k) for A, k in zip(mats, ks))
    flops = sum(2 * A.nnz * k for A, k in zip(mats, ks))
    # error of one member against the FP64 oracle (permuted space)
    j = int(np.argmax([A.nrows for A in mats]))
    rperm, cperm = ctx.get_permutation(hs[j])
    Bo = synth.CSR(mats[j].nrows, mats[j].ncols, *oracle.permute_csr(mats[j], rperm, cperm))
    X = Xs[j].double().cpu().numpy()
    err = oracle.normalized_error(Bo.nrows, Bo.row_ptr, Bo.col, Bo.val, X,
                                  Ys[j].double().cpu().numpy(),
                                  oracle.spmm(Bo.nrows, Bo.row_ptr, Bo.col, Bo.val, X))
    ctx.batch_destroy(plan)
    for h in hs:
        ctx.release(h)
    out = {"matrices": count, "rows": sum(A.nrows for A in mats), "nnz": sum(A.nnz for A in mats),
           "k_mix": {str(k): ks.count(k) for k in sorted(set(ks))}, "us_per_batch": round(us, 1),
           "gbs": round(nb / (us * 1e-6) / 1e9, 1), "gflops": round(flops / (us * 1e-6) / 1e9, 1),
           "bytes_per_batch": nb, "max_normalized_error_sample": err,
           "us_one_launch_per_item_tuned": round(us_items, 1),
           "launch": "one persistent kernel per batch, replayed from a HIP graph"}
    log(f"batch: {out}")
    return out


def serving(ctx_unused, log, pool=32, warm=1000, n_req=20000, low_load_requests=1000):
    import torch
    from paper_2308_00106_amd import mxe as mx
    t = time.perf_counter()
    mats = _generate(synth.serving_member, pool)
    log(f"serving: generated {pool} matrices, {sum(A.nrows for A in mats)} rows, "
        f"{sum(A.nnz for A in mats)} nnz in {time.perf_counter() - t:.1f}s")
    budget = 200 * (1 << 30)
    with mx.Context(0, budget_bytes=budget) as ctx:
        hs = [ctx.permute(ctx.register(A, "f32"), 1000 + i) for i, A in enumerate(mats)]
        Xs = [torch.rand((A.ncols, 8), dtype=torch.float32, device="cuda") * 2 - 1 for A in mats]
        slots = 32
        Ys = [[torch.empty((A.nrows, 8), dtype=torch.float32, device="cuda") for _ in range(slots)]
              for A in mats]
        t = time.perf_counter()
        for h in hs:                        # tune every k class up front
            for k in (1, 2, 4, 8, 16):
                ctx.tune(h, k)
        log(f"serving: tuned {pool} x 5 k classes in {time.perf_counter() - t:.1f}s")
        rng = np.random.default_rng(5)
        # the same product alone, outside the loop: GPU time (events) and the
        # host round trip (launch + synchronize), over random pool requests
        stream = torch.cuda.current_stream()
        alone_gpu, alone_host = [], []
        for _ in range(200):
            m, k = int(rng.integers(0, pool)), int(rng.integers(1, 9))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            th = time.perf_counter()
            e0.record(stream)
            ctx.spmv(hs[m], Xs[m][:, :k], Ys[m][0][:, :k], stream=stream)
            e1.record(stream)
            e1.synchronize()
            alone_host.append((time.perf_counter() - th) * 1e6)
            alone_gpu.append(e0.elapsed_time(e1) * 1e3)
        standalone = {"gpu_p50_us": round(float(np.percentile(alone_gpu, 50)), 1),
                      "host_round_trip_p50_us": round(float(np.percentile(alone_host, 50)), 1),
                      "requests": len(alone_gpu)}
        ctx.serve_start(streams=2, max_inflight=32, max_batch=8, max_merge_k=8)

        def run(rate, n_meas, n_warm, window=256):
            """rate None: closed loop (as fast as possible, at most `window`
            requests outstanding); else open-loop Poisson arrivals."""
            total = n_warm + n_meas
            mi = rng.integers(0, pool, size=total)
            ki = rng.integers(1, 9, size=total)
            nbytes = np.array([_bytes(mats[m], 4, 4, k) for m, k in zip(mi, ki)], dtype=np.float64)
            tickets = [0] * total
            finished = np.zeros(total, dtype=bool)
            lat = np.zeros(total)
            slot_use = [0] * pool
            slot_owner = [[-1] * slots for _ in range(pool)]
            done = threading.Event()

            def waiter():
                for i in range(total):
                    while tickets[i] == 0:
                        time.sleep(0)
                    lat[i] = ctx.wait(tickets[i])
                    finished[i] = True
                done.set()

            wt = threading.Thread(target=waiter)
            wt.start()
            gaps = rng.exponential(1.0 / rate, size=total) if rate else None
            t_next = time.perf_counter()
            t_meas = time.perf_counter()
            n_done = 0
            for i in range(total):
                if i == n_warm:
                    t_meas = time.perf_counter()
                if rate:
                    t_next += gaps[i]
                    while time.perf_counter() < t_next:
                        pass
                else:
                    while i - n_done >= window:
                        while n_done < i and finished[n_done]:
                            n_done += 1
                        time.sleep(0)
                m, k = int(mi[i]), int(ki[i])
                s = slot_use[m] % slots
                slot_use[m] += 1
                owner = slot_owner[m][s]
                while owner >= 0 and not finished[owner]:   # the slot's last writer is done
                    time.sleep(0)
                slot_owner[m][s] = i
                tickets[i] = ctx.submit(hs[m], Xs[m][:, :k], Ys[m][s][:, :k])
            done.wait()
            t1 = time.perf_counter()
            wt.join()
            meas = lat[n_warm:]
            return {"requests": n_meas, "seconds": round(t1 - t_meas, 4),
                    "req_per_s": round(n_meas / (t1 - t_meas), 1),
                    "gbs": round(nbytes[n_warm:].sum() / (t1 - t_meas) / 1e9, 1),
                    "p50_us": round(float(np.percentile(meas, 50)), 1),
                    "p99_us": round(float(np.percentile(meas, 99)), 1),
                    "mean_us": round(float(meas.mean()), 1)}

        closed = run(None, n_req, warm)
        log(f"serving closed loop: {closed}")
        rmax = closed["req_per_s"]
        out = {"pool": pool, "rows": sum(A.nrows for A in mats), "nnz": sum(A.nnz for A in mats),
               "budget_bytes": budget, "closed_loop": closed, "standalone_product": standalone}
        for frac in (0.5, 0.8):
            r = run(frac * rmax, n_req, warm)
            r["offered_req_per_s"] = round(frac * rmax, 1)
            out[f"poisson_{frac}"] = r
            log(f"serving poisson {frac}: {r}")
        low = run(0.05 * rmax, low_load_requests, low_load_requests // 10)
        low["offered_req_per_s"] = round(0.05 * rmax, 1)
        # a served latency runs from submission to the loop seeing the
        # completion, so it holds a launch and a completion check: the host
        # round trip is its like-for-like standalone figure, the GPU time the
        # floor
        low["p50_over_standalone_gpu_p50"] = round(low["p50_us"] / standalone["gpu_p50_us"], 3)
        low["p50_over_standalone_host_p50"] = round(low["p50_us"] / standalone["host_round_trip_p50_us"], 3)
        out["poisson_0.05"] = low
        log(f"serving poisson 0.05: {low}")
        ctx.serve_stop()
    return out


PARTS = {"skewed": skewed, "heavy": heavy, "semiring": semiring, "batch": batch, "serving": serving}


def run_all(ctx, log, parts=tuple(PARTS)):
    return {name: PARTS[name](ctx, log) for name in parts}


def main(argv=None) -> int:
    """`python bench_extras.py [part ...]`: the named parts alone (all by
    default), one JSON line on stdout; used to profile one workload."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("parts", nargs="*", help="any of: " + ", ".join(PARTS))
    args = ap.parse_args(argv)
    unknown = [p for p in args.parts if p not in PARTS]
    if unknown:
        ap.error(f"unknown part(s) {unknown}; choose from {list(PARTS)}")
    args.parts = args.parts or list(PARTS)

    def log(msg):
        print(f"[extras] {msg}", file=sys.stderr, flush=True)

    import torch

    import bench
    from paper_2308_00106_amd import mxe as mx
    ctx = mx.Context(0)
    # first: a 1 GiB read and copy of known size, which also calibrates the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run
    out = {"hbm_ceiling_measured": bench.hbm_ceiling(torch.cuda.current_stream())}
    log(f"hbm ceiling: {out['hbm_ceiling_measured']}")
    out.update(run_all(ctx, log, args.parts))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
