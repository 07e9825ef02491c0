// C ABI of libmxe.so: context, handle table, CSR validation, HBM budget,
// permutation / entropy / SpMV entry points, the SpMV autotuner and batch
// plans captured in HIP graphs. See include/mxe.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <set>

#include "device_common.h"
#include "runtime.h"

namespace mxe {

// ---- errors -------------------------------------------------------------------

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

mxe_status fail(mxe_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

mxe_status hip_fail(hipError_t e, const char *what) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s", what, hipGetErrorString(e));
    set_error(buf);
    return e == hipErrorOutOfMemory ? MXE_ERR_OUT_OF_MEMORY : MXE_ERR_DEVICE;
}

int elem_bytes_of(mxe_dtype d) { return d == MXE_F64 ? 8 : 4; }
static int val_bytes_of(mxe_dtype d) { return d == MXE_F64 ? 8 : d == MXE_F32 ? 4 : 2; }
static int vtype_of(mxe_dtype d) { return d == MXE_F64 ? VAL_F64 : d == MXE_F32 ? VAL_F32 : VAL_BF16; }

namespace {

// Stream-ordered allocation from the device's pool (freed blocks stay cached).
struct Scratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    Scratch() = default;
    Scratch(const Scratch &) = delete;
    ~Scratch() {
        if (p) (void)hipFreeAsync(p, s);
    }
    mxe_status alloc(size_t bytes, hipStream_t stream) {
        s = stream;
        hipError_t e = hipMallocAsync(&p, std::max<size_t>(bytes, 256), stream);
        if (e != hipSuccess) {
            p = nullptr;
            return hip_fail(e, "hipMallocAsync(workspace)");
        }
        return MXE_OK;
    }
};

mxe_status dev_alloc(Matrix &m, void **p, size_t bytes, hipStream_t s) {
    hipError_t e = hipMallocAsync(p, std::max<size_t>(bytes, 256), s);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMallocAsync(matrix)");
    }
    m.allocs.push_back(*p);
    return MXE_OK;
}

uint64_t csr_bytes(int32_t nrows, int64_t nnz, mxe_dtype st) {
    return 4ull * (uint64_t)(nrows + 1) + (uint64_t)nnz * (4ull + (uint64_t)val_bytes_of(st));
}

mxe_status reserve(mxe_ctx *ctx, uint64_t bytes) {
    uint64_t cur = ctx->used.load();
    for (;;) {
        if (ctx->budget && cur + bytes > ctx->budget) {
            char buf[256];
            snprintf(buf, sizeof buf, "HBM budget exceeded: %llu held + %llu requested > %llu",
                     (unsigned long long)cur, (unsigned long long)bytes,
                     (unsigned long long)ctx->budget);
            return fail(MXE_ERR_BUDGET, buf);
        }
        if (ctx->used.compare_exchange_weak(cur, cur + bytes)) return MXE_OK;
    }
}

// When the last reference goes, the work each stream queued on the matrix
// (its last recorded use) finishes before the memory returns to the pool;
// other streams and unrelated work are not waited for.
std::shared_ptr<Matrix> make_matrix(mxe_ctx *ctx) {
    int dev = ctx->device;
    return std::shared_ptr<Matrix>(new Matrix(), [ctx, dev](Matrix *m) {
        DeviceGuard g(dev);
        for (const Matrix::Use &u : m->uses) {
            (void)hipEventSynchronize(u.ev);
            (void)hipEventDestroy(u.ev);
        }
        for (void *p : m->allocs) (void)hipFreeAsync(p, nullptr);
        ctx->used -= m->bytes;
        delete m;
    });
}

int64_t root_of(const Matrix &m) { return m.parent ? m.parent->id : m.id; }

}  // namespace

mxe_status note_use(Matrix &A, hipStream_t s) {
    for (Matrix::Use &u : A.uses)
        if (u.s == s) {
            MXE_HIP(hipEventRecord(u.ev, s));
            return MXE_OK;
        }
    Matrix::Use u{s, nullptr};
    MXE_HIP(hipEventCreateWithFlags(&u.ev, hipEventDisableTiming));
    A.uses.push_back(u);
    MXE_HIP(hipEventRecord(u.ev, s));
    return MXE_OK;
}

std::shared_ptr<Matrix> find_matrix(mxe_ctx *ctx, mxe_mat h) {
    auto it = ctx->mats.find(h);
    return it == ctx->mats.end() ? nullptr : it->second;
}

uint64_t request_bytes(const Matrix &A, int32_t k) {
    return csr_bytes(A.nrows, A.nnz, A.storage) +
           (uint64_t)k * ((uint64_t)A.ncols + A.nrows) * elem_bytes_of(A.storage);
}

// ---- row bins and merge workspace (built once per matrix) -------------------------

static mxe_status ensure_bins(mxe_ctx *, Matrix &A, hipStream_t s) {
    if (A.bins_ready) return MXE_OK;
    void *p;
    mxe_status st = dev_alloc(A, &p, sizeof(int32_t) * ((size_t)A.nrows + 1), s);
    if (st) return st;
    A.bin_list = (int32_t *)p;
    st = dev_alloc(A, &p, sizeof(int32_t) * (kNumBins + 2), s);
    if (st) return st;
    A.bin_off_dev = (int32_t *)p;
    Scratch ws;
    if ((st = ws.alloc(row_bins_ws_bytes(A.nrows), s))) return st;
    MXE_HIP(launch_row_bins(A.nrows, A.rp, A.bin_list, A.bin_off_dev, ws.p, s));
    MXE_HIP(launch_row_max(A.nrows, A.rp, A.bin_off_dev + kNumBins + 1, s));
    int32_t host[kNumBins + 2];
    MXE_HIP(hipMemcpyAsync(host, A.bin_off_dev, sizeof host, hipMemcpyDeviceToHost, s));
    MXE_HIP(hipStreamSynchronize(s));
    std::memcpy(A.bin_off, host, sizeof A.bin_off);
    A.max_row = host[kNumBins + 1];
    A.bins_ready = true;
    return MXE_OK;
}

// Structures built once per matrix on the calling stream are finished
// (the stream synchronized) before any launch uses them, so a launch on
// another stream never reads one half built; afterwards they are read only.

// merge-path slice starts (built once per matrix)
static mxe_status ensure_merge(mxe_ctx *ctx, Matrix &A, hipStream_t s) {
    if (A.merge_coords) return MXE_OK;
    const uint64_t bytes = merge_coords_bytes(A.nrows, A.nnz);
    mxe_status st;
    if ((st = reserve(ctx, bytes))) return st;
    A.bytes += bytes;
    void *p;
    if ((st = dev_alloc(A, &p, bytes, s))) return st;
    MXE_HIP(launch_merge_coords(A.nrows, A.nnz, A.rp, p, s));
    MXE_HIP(hipStreamSynchronize(s));
    A.merge_coords = p;
    return MXE_OK;
}

// COO row index per entry (built once per matrix)
static mxe_status ensure_coo(mxe_ctx *ctx, Matrix &A, hipStream_t s) {
    if (A.coo_row) return MXE_OK;
    const uint64_t bytes = 4ull * (uint64_t)A.nnz;
    mxe_status st;
    if ((st = reserve(ctx, bytes))) return st;
    A.bytes += bytes;
    void *r;
    if ((st = dev_alloc(A, &r, 4 * (size_t)A.nnz, s))) return st;
    MXE_HIP(launch_coo_rows(A.nrows, A.rp, (int32_t *)r, s));
    MXE_HIP(hipStreamSynchronize(s));
    A.coo_row = (int32_t *)r;
    return MXE_OK;
}

static int kclass_of(int32_t k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16; }

static SpmvArgs make_args(Matrix &A, int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy) {
    SpmvArgs a{};
    a.nrows = A.nrows;
    a.ncols = A.ncols;
    a.nnz = A.nnz;
    a.rp = A.rp;
    a.col = A.col;
    a.val = A.val;
    a.vtype = vtype_of(A.storage);
    a.k = k;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.bin_list = A.bin_list;
    a.bin_off_host = A.bin_off;
    a.merge_coords = A.merge_coords;
    a.coo_row = A.coo_row;
    return a;
}

// bytes of the launch's own carry workspace: MERGE and COO, else 0
static size_t carry_bytes(const Matrix &A, int variant, int32_t k) {
    const int family = variant & 0xf00;
    if (family == MXE_VAR_MERGE) return merge_carry_bytes(A.nrows, A.nnz);
    if (family == MXE_VAR_COO) return coo_ws_bytes(A.nnz, kclass_of(k), elem_bytes_of(A.storage));
    return 0;
}

static TuneKey tune_key(const Matrix &A, int32_t k) {
    return TuneKey{A.nrows, A.ncols, A.nnz, (int32_t)A.storage, kclass_of(k),
                   A.seed, A.mode, root_of(A)};
}

// ---- column-slab layouts (built once per matrix, k class and slab size) ----------

// slab size: `units` x 64 KiB of x
static int64_t slab_bytes_of(int units) { return (int64_t)units << 16; }
// a SLAB variant's slab size and the CUs its row blocks are sized for (two
// workgroups per CU; MXE_SLAB_ONE_PER_CU: one, so blocks for half the CUs)
static int slab_units_of(int variant) { return variant & (MXE_SLAB_ONE_PER_CU - 1); }
static int slab_cus_of(const mxe_ctx *ctx, int variant) {
    return (variant & MXE_SLAB_ONE_PER_CU) ? std::max(1, ctx->cu_count / 2) : ctx->cu_count;
}

// LDS a slab layout gives a block's partial y: half the CU's LDS, so two
// workgroups of any layout fit on a CU (the batch kernel runs two per CU),
// less 8 KiB for the kernels' own arrays and the allocation granule.
static int64_t slab_y_lds(const mxe_ctx *ctx) {
    return std::min<int64_t>((int64_t)ctx->lds_per_cu / 2, (int64_t)ctx->lds_per_block) - 8 * 1024;
}

// Blocks of a single product's layout that run at once: two per CU of the
// device. A batch's per-XCD layouts (sized for one XCD's CUs) feed work
// queues instead, where the largest blocks are best: 0.
static int64_t slab_resident(const mxe_ctx *ctx, int cus) {
    const int xcd_cus = std::max(1, ctx->cu_count / kBatchQueues);
    return cus == xcd_cus ? 0 : 2 * (int64_t)ctx->cu_count;
}

static bool layout_geometry(const mxe_ctx *ctx, const Matrix &A, int kclass, int units, int cus,
                            SlabGeom *g) {
    return slab_geometry(A.nrows, A.ncols, kclass, vtype_of(A.storage), cus, slab_bytes_of(units),
                         slab_y_lds(ctx), slab_resident(ctx, cus), g);
}

// cus: the compute units whose workgroups share the matrix, which sizes the
// row blocks (all of the device for a single product, one XCD's in a batch)
static mxe_status ensure_slab(mxe_ctx *ctx, Matrix &A, int kclass, int units, int cus,
                              hipStream_t s, const Matrix::Slab **out) {
    const auto key = std::make_tuple(kclass, units, cus);
    auto it = A.slabs.find(key);
    if (it != A.slabs.end()) {
        *out = &it->second;
        return MXE_OK;
    }
    Matrix::Slab sl;
    if (!layout_geometry(ctx, A, kclass, units, cus, &sl.g))
        return fail(MXE_ERR_UNSUPPORTED, "column-slab layout does not fit this matrix");
    const int vb = val_bytes_of(A.storage);
    const size_t noff = slab_offsets_count(sl.g);
    const uint64_t bytes = 4ull * noff + (uint64_t)A.nnz * (4ull + vb);
    mxe_status st;
    if ((st = reserve(ctx, bytes))) return st;
    A.bytes += bytes;
    void *p;
    if ((st = dev_alloc(A, &p, 4 * noff, s))) return st;
    sl.off = (int32_t *)p;
    if ((st = dev_alloc(A, &p, 4 * (size_t)A.nnz, s))) return st;
    sl.idx = (uint32_t *)p;
    if ((st = dev_alloc(A, &p, (size_t)vb * A.nnz, s))) return st;
    sl.val = p;
    Scratch ws;
    if ((st = ws.alloc(slab_build_ws_bytes(sl.g), s))) return st;
    MXE_HIP(launch_slab_build(sl.g, A.rp, A.col, A.val, vb, sl.off, sl.idx, sl.val, ws.p, s));
    MXE_HIP(hipStreamSynchronize(s));
    *out = &(A.slabs[key] = sl);
    return MXE_OK;
}

static void drop_slab(mxe_ctx *ctx, Matrix &A, const Matrix::Slab &sl, hipStream_t s) {
    uint64_t bytes = 4ull * slab_offsets_count(sl.g) +
                     (uint64_t)A.nnz * (4ull + (uint64_t)val_bytes_of(A.storage));
    if (sl.wstart) bytes += 4ull * sl.g.blocks;
    for (void *p : {(void *)sl.off, (void *)sl.idx, sl.val, (void *)sl.wstart}) {
        if (!p) continue;
        A.allocs.erase(std::remove(A.allocs.begin(), A.allocs.end(), p), A.allocs.end());
        (void)hipFreeAsync(p, s);
    }
    A.bytes -= bytes;
    ctx->used -= bytes;
}

// Rows of x (columns of the matrix) the LDS window of a block of layout g
// holds: what a workgroup's share of its CU's LDS leaves beside the block's
// partial y and the kernel's own arrays, at most 128 KiB; 0 when under 256.
static int32_t window_rows(const mxe_ctx *ctx, const SlabGeom &g, int eb) {
    const int64_t per_cu = std::max<int64_t>(1, (g.blocks + ctx->cu_count - 1) / ctx->cu_count);
    const int64_t share = std::min<int64_t>((int64_t)ctx->lds_per_cu / per_cu, (int64_t)ctx->lds_per_block);
    const int64_t avail = share - 8 * 1024 - (int64_t)slab_window_offset(g, eb);
    const int64_t rows = std::min<int64_t>(avail, 128 * 1024) / ((int64_t)g.kclass * eb);
    if (rows < 256) return 0;
    return (int32_t)std::min<int64_t>(rows, g.ncols);
}

// MXE_VAR_WINDOW: the layout's per-block window starts, built once.
static mxe_status ensure_window(mxe_ctx *ctx, Matrix &A, Matrix::Slab &sl, hipStream_t s) {
    if (sl.wstart) return MXE_OK;
    const int32_t win = window_rows(ctx, sl.g, elem_bytes_of(A.storage));
    if (win < 1) return fail(MXE_ERR_UNSUPPORTED, "no LDS left for an x window in this layout");
    const uint64_t bytes = 4ull * sl.g.blocks;
    mxe_status st;
    if ((st = reserve(ctx, bytes))) return st;
    A.bytes += bytes;
    void *p;
    if ((st = dev_alloc(A, &p, bytes, s))) return st;
    MXE_HIP(launch_slab_window(sl.g, A.rp, A.col, win, (int32_t *)p, s));
    MXE_HIP(hipStreamSynchronize(s));
    sl.wstart = (int32_t *)p;
    sl.win = win;
    return MXE_OK;
}

static bool slab_family(int variant) {
    return (variant & 0xf00) == MXE_VAR_SLAB || (variant & 0xf00) == MXE_VAR_WINDOW;
}

// Arguments for one launch of `variant`, building what the variant needs.
static mxe_status prepare_args(mxe_ctx *ctx, Matrix &A, int variant, int32_t k, const void *X,
                               int64_t ldx, void *Y, int64_t ldy, hipStream_t s, SpmvArgs *a) {
    const int family = variant & 0xf00;
    mxe_status st;
    if (family == MXE_VAR_BINNED && (st = ensure_bins(ctx, A, s))) return st;
    if (family == MXE_VAR_MERGE && (st = ensure_merge(ctx, A, s))) return st;
    if (family == MXE_VAR_COO && (st = ensure_coo(ctx, A, s))) return st;
    *a = make_args(A, k, X, ldx, Y, ldy);
    if (slab_family(variant)) {
        const Matrix::Slab *sl;
        if ((st = ensure_slab(ctx, A, kclass_of(k), slab_units_of(variant), slab_cus_of(ctx, variant),
                              s, &sl)))
            return st;
        a->slab = &sl->g;
        a->slab_off = sl->off;
        a->slab_idx = sl->idx;
        a->slab_val = sl->val;
        if (family == MXE_VAR_WINDOW) {
            Matrix::Slab &w = const_cast<Matrix::Slab &>(*sl);
            if ((st = ensure_window(ctx, A, w, s))) return st;
            a->slab_wstart = w.wstart;
            a->slab_win = w.win;
        }
    }
    return MXE_OK;
}

// ---- autotuner ---------------------------------------------------------------------
// Times every variant (GROUP with 1..64 lanes, BINNED, FIXED, MERGE when
// k <= 4, SLAB with 0.75, 1, 2 and 4 MiB slabs at two workgroups per CU and
// 1, 1.25 and 1.5 MiB at one, when the layout fits) on the matrix itself
// with scratch vectors, times the fastest few again and keeps the winner;
// also keeps the fastest GROUP lanes for the persistent batch kernel.
static mxe_status tune(mxe_ctx *ctx, Matrix &A, int32_t k, hipStream_t s, TuneResult *out) {
    mxe_status st;
    const int kc = kclass_of(k);
    const size_t eb = elem_bytes_of(A.storage);
    Scratch xs, ys;
    if ((st = xs.alloc(eb * (size_t)std::max(A.ncols, 1) * kc, s))) return st;
    if ((st = ys.alloc(eb * (size_t)std::max(A.nrows, 1) * kc, s))) return st;
    MXE_HIP(hipMemsetAsync(xs.p, 0, eb * (size_t)std::max(A.ncols, 1) * kc, s));
    std::vector<int> cands;
    for (int l = 1; l <= 64; l <<= 1) cands.push_back(MXE_VARIANT(MXE_VAR_GROUP, l));
    cands.push_back(MXE_VARIANT(MXE_VAR_BINNED, 0));
    cands.push_back(MXE_VARIANT(MXE_VAR_FIXED, std::max(kc, 8)));
    if (kc <= 4) cands.push_back(MXE_VARIANT(MXE_VAR_MERGE, 0));
    // 0.75, 1, 2 and 4 MiB of x per slab with two workgroups per CU; 1, 1.25
    // and 1.5 MiB with one (each workgroup then walks twice the rows per slab)
    for (int units : {12, 16, 32, 64, 16 | MXE_SLAB_ONE_PER_CU, 20 | MXE_SLAB_ONE_PER_CU,
                      24 | MXE_SLAB_ONE_PER_CU}) {
        const int v = MXE_VARIANT(MXE_VAR_SLAB, units);
        SlabGeom g;
        if (layout_geometry(ctx, A, kc, slab_units_of(v), slab_cus_of(ctx, v), &g))
            cands.push_back(v);
    }
    // the same layouts with an LDS window of x per row block (one workgroup
    // per CU leaves the widest window; two per CU, a narrower one)
    for (int units : {16 | MXE_SLAB_ONE_PER_CU, 32 | MXE_SLAB_ONE_PER_CU, 32}) {
        const int v = MXE_VARIANT(MXE_VAR_WINDOW, units);
        SlabGeom g;
        if (layout_geometry(ctx, A, kc, slab_units_of(v), slab_cus_of(ctx, v), &g) &&
            window_rows(ctx, g, (int)eb) > 0)
            cands.push_back(v);
    }
    std::set<std::tuple<int, int, int>> had;          // layouts other work may be using
    for (const auto &kv : A.slabs) had.insert(kv.first);
    hipEvent_t e0, e1;
    MXE_HIP(hipEventCreate(&e0));
    MXE_HIP(hipEventCreate(&e1));
    // milliseconds per product of variant v over reps launches after a warm-up
    auto time_variant = [&](int v, int reps, float *per) -> mxe_status {
        SpmvArgs a;
        mxe_status st2 = prepare_args(ctx, A, v, kc, xs.p, kc, ys.p, kc, s, &a);
        if (st2) return st2;
        Scratch cw;
        if (const size_t cb = carry_bytes(A, v, kc)) {
            if ((st2 = cw.alloc(cb, s))) return st2;
            a.carry_ws = cw.p;
        }
        hipError_t e = launch_spmv(a, v, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_spmv(a, v, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) return hip_fail(e, "autotune");
        *per = ms / reps;
        return MXE_OK;
    };
    // stage 1: every candidate, briefly
    const int reps = A.nnz > 4000000 ? 3 : 10;
    std::vector<std::pair<float, int>> timed;            // (ms per product, variant)
    float best_group = std::numeric_limits<float>::max();
    TuneResult r{cands[0], 1};
    mxe_status result = MXE_OK;
    for (int v : cands) {
        float ms = 0;
        if ((result = time_variant(v, reps, &ms))) {
            // a layout that does not fit the matrix or the HBM budget is not a candidate
            if (result == MXE_ERR_UNSUPPORTED || result == MXE_ERR_BUDGET) {
                result = MXE_OK;
                continue;
            }
            break;
        }
        if (getenv("MXE_LOG"))
            fprintf(stderr, "[mxe] tune rows=%d nnz=%lld k=%d variant 0x%x: %.2f us\n", A.nrows,
                    (long long)A.nnz, kc, v, 1e3f * ms);
        timed.push_back({ms, v});
        // the persistent batch kernel runs multi-RHS items with lanes >= k class
        if ((v & 0xf00) == MXE_VAR_GROUP && (v & 0xff) >= kc && ms < best_group) {
            best_group = ms;
            r.group_lanes = v & 0xff;
        }
    }
    // stage 2: the candidates within 8% of the fastest (two to five of them)
    // again, interleaved over two rounds of 10 products each, so candidates a
    // few percent apart are told apart
    if (result == MXE_OK && !timed.empty()) {
        std::stable_sort(timed.begin(), timed.end());
        size_t top = 1;
        while (top < timed.size() && top < 5 &&
               (top < 2 || timed[top].first <= 1.08f * timed[0].first))
            ++top;
        std::vector<float> total(top, 0.0f);
        for (int round = 0; round < 2 && result == MXE_OK; ++round)
            for (size_t i = 0; i < top && result == MXE_OK; ++i) {
                float ms = 0;
                if ((result = time_variant(timed[i].second, 10, &ms)) == MXE_OK) total[i] += ms;
            }
        if (result == MXE_OK) {
            const size_t b = std::min_element(total.begin(), total.end()) - total.begin();
            r.variant = timed[b].second;
            if (getenv("MXE_LOG"))
                fprintf(stderr, "[mxe] tune rows=%d k=%d chose 0x%x: %.2f us\n", A.nrows, kc,
                        r.variant, 1e3f * total[b] / 2);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // column-slab layouts built here for this k class and not chosen are freed
    // (stream-ordered after the timing launches)
    for (auto it = A.slabs.begin(); it != A.slabs.end();) {
        const bool chosen = result == MXE_OK && slab_family(r.variant) &&
                            std::get<1>(it->first) == slab_units_of(r.variant) &&
                            std::get<2>(it->first) == slab_cus_of(ctx, r.variant);
        if (std::get<0>(it->first) == kc && !had.count(it->first) && !chosen) {
            drop_slab(ctx, A, it->second, s);
            it = A.slabs.erase(it);
        } else {
            ++it;
        }
    }
    if (result != MXE_OK) return result;
    ctx->tuned[tune_key(A, k)] = r;
    if (out) *out = r;
    return MXE_OK;
}

mxe_status ensure_variant(mxe_ctx *ctx, Matrix &A, int32_t k, hipStream_t s, TuneResult *out) {
    auto it = ctx->tuned.find(tune_key(A, k));
    if (it != ctx->tuned.end()) {
        *out = it->second;
        return MXE_OK;
    }
    return tune(ctx, A, k, s, out);
}

// ---- products -------------------------------------------------------------------------

static mxe_status spmv_core(mxe_ctx *ctx, Matrix &A, int32_t k, const void *X, int64_t ldx,
                            void *Y, int64_t ldy, hipStream_t s) {
    const int eb = elem_bytes_of(A.storage);
    for (int32_t c0 = 0; c0 < k; c0 += 16) {
        const int32_t kc = std::min<int32_t>(16, k - c0);
        TuneResult r;
        mxe_status st = ensure_variant(ctx, A, kc, s, &r);
        if (st) return st;
        SpmvArgs a;
        if ((st = prepare_args(ctx, A, r.variant, kc, (const char *)X + (size_t)c0 * eb, ldx,
                               (char *)Y + (size_t)c0 * eb, ldy, s, &a)))
            return st;
        Scratch cw;                             // this launch's carries (MERGE, COO)
        if (const size_t cb = carry_bytes(A, r.variant, kc)) {
            if ((st = cw.alloc(cb, s))) return st;
            a.carry_ws = cw.p;
        }
        MXE_HIP(launch_spmv(a, r.variant, s));
    }
    return MXE_OK;
}

mxe_status spmv_internal(mxe_ctx *ctx, Matrix &A, int32_t k, const void *X, int64_t ldx, void *Y,
                         int64_t ldy, uint32_t flags, hipStream_t s) {
    if (!(flags & MXE_SPACE_ORIGINAL) || !A.rperm) {
        mxe_status st = spmv_core(ctx, A, k, X, ldx, Y, ldy, s);
        return st ? st : note_use(A, s);
    }
    // Eq. 1: y = P_r^-1 (B (P_c^-1 x))
    const int eb = elem_bytes_of(A.storage);
    Scratch xp, yp;
    mxe_status st;
    if ((st = xp.alloc((size_t)eb * std::max(A.ncols, 1) * k, s))) return st;
    if ((st = yp.alloc((size_t)eb * std::max(A.nrows, 1) * k, s))) return st;
    MXE_HIP(launch_gather_rows(A.ncols, k, A.cperm, X, ldx, xp.p, k, eb, s));
    if ((st = spmv_core(ctx, A, k, xp.p, k, yp.p, k, s))) return st;
    MXE_HIP(launch_scatter_rows(A.nrows, k, A.rperm, yp.p, k, Y, ldy, eb, s));
    return note_use(A, s);
}

}  // namespace mxe

using namespace mxe;

// ============================== C ABI ==========================================

extern "C" {

const char *mxe_status_string(mxe_status s) {
    switch (s) {
    case MXE_OK: return "ok";
    case MXE_ERR_INVALID_ARG: return "invalid argument";
    case MXE_ERR_INVALID_CSR: return "invalid CSR";
    case MXE_ERR_NOT_FOUND: return "handle not found";
    case MXE_ERR_BUSY: return "busy";
    case MXE_ERR_BUDGET: return "HBM budget exceeded";
    case MXE_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MXE_ERR_UNSUPPORTED: return "unsupported";
    case MXE_ERR_TIMEOUT: return "timeout";
    case MXE_ERR_DEVICE: return "device error";
    case MXE_ERR_INEXACT: return "rounding not certified";
    }
    return "unknown status";
}

const char *mxe_last_error(void) { return g_last_error.c_str(); }

int32_t mxe_abi_version(void) { return MXE_ABI_VERSION; }

mxe_status mxe_validate_csr(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx) {
    if (nrows < 0 || ncols < 0 || nnz < 0 || nnz > INT32_MAX)
        return fail(MXE_ERR_INVALID_ARG, "negative size or nnz >= 2^31");
    if (!row_ptr || (nnz > 0 && !col_idx)) return fail(MXE_ERR_INVALID_ARG, "NULL array");
    if (nnz > 0 && (nrows == 0 || ncols == 0))
        return fail(MXE_ERR_INVALID_CSR, "entries in an empty shape");
    if (row_ptr[0] != 0) return fail(MXE_ERR_INVALID_CSR, "row_ptr[0] != 0");
    if (row_ptr[nrows] != nnz) return fail(MXE_ERR_INVALID_CSR, "row_ptr[nrows] != nnz");
    for (int32_t i = 0; i < nrows; ++i) {
        const int32_t a = row_ptr[i], b = row_ptr[i + 1];
        if (b < a) {
            char buf[128];
            snprintf(buf, sizeof buf, "row_ptr decreases at row %d", i);
            return fail(MXE_ERR_INVALID_CSR, buf);
        }
        if (b > nnz) return fail(MXE_ERR_INVALID_CSR, "row_ptr exceeds nnz");
        for (int32_t e = a; e < b; ++e) {
            const int32_t c = col_idx[e];
            if (c < 0 || c >= ncols) {
                char buf[128];
                snprintf(buf, sizeof buf, "column %d out of range in row %d", c, i);
                return fail(MXE_ERR_INVALID_CSR, buf);
            }
            if (e > a && c <= col_idx[e - 1]) {
                char buf[128];
                snprintf(buf, sizeof buf, "columns not strictly increasing in row %d", i);
                return fail(MXE_ERR_INVALID_CSR, buf);
            }
        }
    }
    return MXE_OK;
}

mxe_status mxe_create(int32_t device, uint64_t hbm_budget_bytes, mxe_ctx **out) {
    if (!out) return fail(MXE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0)
        return fail(MXE_ERR_DEVICE, "no HIP device");
    if (device < 0 || device >= n) return fail(MXE_ERR_INVALID_ARG, "device index out of range");
    hipDeviceProp_t prop;
    MXE_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MXE_ERR_DEVICE, std::string("not a gfx950 device: ") + prop.gcnArchName);
    DeviceGuard g(device);
    hipMemPool_t pool;
    MXE_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t thr = UINT64_MAX;
    MXE_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    mxe_status st = noalloc_init(device);
    if (st) return st;
    auto *ctx = new mxe_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    ctx->cu_count = prop.multiProcessorCount;
    ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    ctx->lds_per_block = prop.sharedMemPerBlock;
    *out = ctx;
    return MXE_OK;
}

mxe_status mxe_destroy(mxe_ctx *ctx) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    serve_destroy(ctx);
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        ctx->plans.clear();
        ctx->mats.clear();
    }
    delete ctx;
    return MXE_OK;
}

mxe_status mxe_register_matrix(mxe_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz,
                               const int32_t *row_ptr, const int32_t *col_idx, const double *vals,
                               mxe_dtype storage, uint32_t flags, mxe_mat *out) {
    if (!ctx || !out) return fail(MXE_ERR_INVALID_ARG, "ctx or out is NULL");
    if (storage != MXE_F64 && storage != MXE_F32 && storage != MXE_BF16)
        return fail(MXE_ERR_INVALID_ARG, "unknown storage dtype");
    if (flags & ~MXE_INPUT_DEVICE) return fail(MXE_ERR_INVALID_ARG, "unknown flags");
    if (nrows < 0 || ncols < 0 || nnz < 0 || nnz > INT32_MAX)
        return fail(MXE_ERR_INVALID_ARG, "negative size or nnz >= 2^31");
    if (!row_ptr || (nnz > 0 && (!col_idx || !vals))) return fail(MXE_ERR_INVALID_ARG, "NULL array");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    const bool on_dev = flags & MXE_INPUT_DEVICE;
    mxe_status st;
    std::vector<int32_t> hrp, hcol;
    const int32_t *vrp = row_ptr, *vcol = col_idx;
    if (on_dev) {               // validate a host staging copy
        hrp.resize((size_t)nrows + 1);
        hcol.resize((size_t)nnz);
        MXE_HIP(hipMemcpy(hrp.data(), row_ptr, 4 * hrp.size(), hipMemcpyDeviceToHost));
        if (nnz) MXE_HIP(hipMemcpy(hcol.data(), col_idx, 4 * hcol.size(), hipMemcpyDeviceToHost));
        vrp = hrp.data();
        vcol = hcol.data();
    }
    if ((st = mxe_validate_csr(nrows, ncols, nnz, vrp, vcol))) return st;
    auto A = make_matrix(ctx);
    A->nrows = nrows;
    A->ncols = ncols;
    A->nnz = nnz;
    A->storage = storage;
    const uint64_t bytes = csr_bytes(nrows, nnz, storage);
    if ((st = reserve(ctx, bytes))) return st;
    A->bytes = bytes;
    hipStream_t s = nullptr;
    void *p;
    if ((st = dev_alloc(*A, &p, 4 * ((size_t)nrows + 1), s))) return st;
    A->rp = (int32_t *)p;
    if ((st = dev_alloc(*A, &p, 4 * (size_t)nnz, s))) return st;
    A->col = (int32_t *)p;
    if ((st = dev_alloc(*A, &p, (size_t)val_bytes_of(storage) * nnz, s))) return st;
    A->val = p;
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    MXE_HIP(hipMemcpyAsync(A->rp, row_ptr, 4 * ((size_t)nrows + 1), kind, s));
    if (nnz) {
        MXE_HIP(hipMemcpyAsync(A->col, col_idx, 4 * (size_t)nnz, kind, s));
        if (storage == MXE_F64) {
            MXE_HIP(hipMemcpyAsync(A->val, vals, 8 * (size_t)nnz, kind, s));
        } else {
            Scratch tmp;
            if ((st = tmp.alloc(8 * (size_t)nnz, s))) return st;
            MXE_HIP(hipMemcpyAsync(tmp.p, vals, 8 * (size_t)nnz, kind, s));
            MXE_HIP(launch_convert_f64((const double *)tmp.p, A->val, nnz, vtype_of(storage), s));
        }
    }
    MXE_HIP(hipStreamSynchronize(s));
    A->id = ctx->next_id++;
    ctx->mats[A->id] = A;
    *out = A->id;
    return MXE_OK;
}

// per-line nonzero counts ahead of the gradient shuffle's own workspace
static size_t counts_bytes(int64_t n) { return (4 * ((size_t)n + 64) + 255) & ~size_t(255); }

mxe_status mxe_permute(mxe_ctx *ctx, mxe_mat a, uint64_t seed, uint32_t mode, void *stream,
                       mxe_mat *out_b) {
    if (!ctx || !out_b) return fail(MXE_ERR_INVALID_ARG, "ctx or out_b is NULL");
    if (mode & ~(MXE_ROWS | MXE_COLS | MXE_GRADIENT)) return fail(MXE_ERR_INVALID_ARG, "unknown mode bits");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, a);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    hipStream_t s = (hipStream_t)stream;
    const int32_t M = A->nrows, N = A->ncols;
    const uint64_t bytes = csr_bytes(M, A->nnz, A->storage) + 8ull * M + 8ull * N;
    mxe_status st;
    if ((st = reserve(ctx, bytes))) return st;
    auto B = make_matrix(ctx);
    B->bytes = bytes;
    B->nrows = M;
    B->ncols = N;
    B->nnz = A->nnz;
    B->storage = A->storage;
    B->parent = A;
    B->seed = seed;
    B->mode = mode;
    void *p;
    const int vb = val_bytes_of(A->storage);
    if ((st = dev_alloc(*B, &p, 4 * ((size_t)M + 1), s))) return st;
    B->rp = (int32_t *)p;
    if ((st = dev_alloc(*B, &p, 4 * (size_t)A->nnz, s))) return st;
    B->col = (int32_t *)p;
    if ((st = dev_alloc(*B, &p, (size_t)vb * A->nnz, s))) return st;
    B->val = p;
    if ((st = dev_alloc(*B, &p, 4 * (size_t)M, s))) return st;
    B->rperm = (int32_t *)p;
    if ((st = dev_alloc(*B, &p, 4 * (size_t)M, s))) return st;
    B->rinv = (int32_t *)p;
    if ((st = dev_alloc(*B, &p, 4 * (size_t)N, s))) return st;
    B->cperm = (int32_t *)p;
    if ((st = dev_alloc(*B, &p, 4 * (size_t)N, s))) return st;
    B->cinv = (int32_t *)p;
    // stream seeds: first and second SplitMix64 outputs started at `seed`
    const uint64_t s_row = sm64_key(seed, 0), s_col = sm64_key(seed, 1);
    Scratch ws;
    const bool grad = mode & MXE_GRADIENT;
    size_t ws_bytes = std::max({random_perm_ws_bytes(M), random_perm_ws_bytes(N),
                                permuted_row_ptr_ws_bytes(M)});
    if (grad)
        ws_bytes = std::max({ws_bytes, gradient_perm_ws_bytes(M) + counts_bytes(M),
                             gradient_perm_ws_bytes(N) + counts_bytes(N)});
    if ((st = ws.alloc(ws_bytes, s))) return st;
    // gradient formats (Section 8, G-R and G-C): per-line counts go first in
    // the workspace, the shuffle's own workspace after them
    auto gradient = [&](bool rows, int32_t n, uint64_t seed_n, int32_t *perm, int32_t *inv) {
        int32_t *counts = (int32_t *)ws.p;
        void *gws = (char *)ws.p + counts_bytes(n);
        hipError_t e = launch_line_counts(rows, M, A->nnz, A->rp, A->col, n, counts, s);
        if (e == hipSuccess) e = launch_gradient_perm(n, counts, seed_n, perm, inv, gws, s);
        return e;
    };
    if ((mode & MXE_ROWS) && grad) {
        MXE_HIP(gradient(true, M, s_row, B->rperm, B->rinv));
    } else if (mode & MXE_ROWS) {
        MXE_HIP(launch_random_perm(M, s_row, B->rperm, B->rinv, ws.p, s));
    } else {
        MXE_HIP(launch_iota_i32(B->rperm, M, s));
        MXE_HIP(launch_iota_i32(B->rinv, M, s));
    }
    if ((mode & MXE_COLS) && grad) {
        MXE_HIP(gradient(false, N, s_col, B->cperm, B->cinv));
    } else if (mode & MXE_COLS) {
        MXE_HIP(launch_random_perm(N, s_col, B->cperm, B->cinv, ws.p, s));
    } else {
        MXE_HIP(launch_iota_i32(B->cperm, N, s));
        MXE_HIP(launch_iota_i32(B->cinv, N, s));
    }
    MXE_HIP(launch_permuted_row_ptr(M, A->rp, B->rperm, B->rp, ws.p, s));
    MXE_HIP(launch_gather_relabel_sort(M, A->rp, A->col, A->val, vb, B->rinv,
                                       (mode & MXE_COLS) ? B->cinv : nullptr, B->rp, B->col,
                                       B->val, s));
    if ((st = note_use(*A, s)) || (st = note_use(*B, s))) return st;
    B->id = ctx->next_id++;
    ctx->mats[B->id] = B;
    *out_b = B->id;
    return MXE_OK;
}

mxe_status mxe_get_permutation(mxe_ctx *ctx, mxe_mat b, int32_t *rperm, int32_t *cperm,
                               uint32_t flags, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto B = find_matrix(ctx, b);
    if (!B) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = (flags & MXE_OUTPUT_DEVICE) ? hipMemcpyDeviceToDevice
                                                           : hipMemcpyDeviceToHost;
    if (B->rperm) {
        if (rperm && B->nrows) MXE_HIP(hipMemcpyAsync(rperm, B->rperm, 4 * (size_t)B->nrows, kind, s));
        if (cperm && B->ncols) MXE_HIP(hipMemcpyAsync(cperm, B->cperm, 4 * (size_t)B->ncols, kind, s));
    } else {
        if (flags & MXE_OUTPUT_DEVICE) {
            if (rperm) MXE_HIP(launch_iota_i32(rperm, B->nrows, s));
            if (cperm) MXE_HIP(launch_iota_i32(cperm, B->ncols, s));
        } else {
            if (rperm) for (int32_t i = 0; i < B->nrows; ++i) rperm[i] = i;
            if (cperm) for (int32_t i = 0; i < B->ncols; ++i) cperm[i] = i;
        }
    }
    MXE_HIP(hipStreamSynchronize(s));
    return MXE_OK;
}

mxe_status mxe_export_csr(mxe_ctx *ctx, mxe_mat m, int32_t *row_ptr, int32_t *col_idx, void *vals,
                          uint32_t flags, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = (flags & MXE_OUTPUT_DEVICE) ? hipMemcpyDeviceToDevice
                                                           : hipMemcpyDeviceToHost;
    if (row_ptr) MXE_HIP(hipMemcpyAsync(row_ptr, A->rp, 4 * ((size_t)A->nrows + 1), kind, s));
    if (col_idx && A->nnz) MXE_HIP(hipMemcpyAsync(col_idx, A->col, 4 * (size_t)A->nnz, kind, s));
    if (vals && A->nnz)
        MXE_HIP(hipMemcpyAsync(vals, A->val, (size_t)val_bytes_of(A->storage) * A->nnz, kind, s));
    MXE_HIP(hipStreamSynchronize(s));
    return MXE_OK;
}

mxe_status mxe_matrix_info(mxe_ctx *ctx, mxe_mat m, mxe_matrix_desc *out) {
    if (!ctx || !out) return fail(MXE_ERR_INVALID_ARG, "ctx or out is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    mxe_status st = ensure_bins(ctx, *A, nullptr);
    if (st) return st;
    out->nrows = A->nrows;
    out->ncols = A->ncols;
    out->nnz = A->nnz;
    out->storage = A->storage;
    out->permuted = A->parent ? 1 : 0;
    out->parent = A->parent ? A->parent->id : 0;
    out->seed = A->seed;
    out->mode = A->mode;
    out->device_bytes = A->bytes;
    out->max_row = A->max_row;
    out->mean_row = A->nrows ? (double)A->nnz / A->nrows : 0.0;
    return MXE_OK;
}

mxe_status mxe_release(mxe_ctx *ctx, mxe_mat m) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->mats.find(m);
    if (it == ctx->mats.end()) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    if (it->second->busy.load() > 0) return fail(MXE_ERR_BUSY, "matrix has serving work in flight");
    ctx->mats.erase(it);
    return MXE_OK;
}

mxe_status mxe_entropy(mxe_ctx *ctx, mxe_mat m, int32_t grid_rows, int32_t grid_cols,
                       void *stream, double *h_bits, double *h_nats, int64_t *hist) {
    if (!ctx || !h_bits) return fail(MXE_ERR_INVALID_ARG, "ctx or h_bits is NULL");
    if (grid_rows < 1 || grid_cols < 1 || grid_rows > (1 << 20) || grid_cols > (1 << 20))
        return fail(MXE_ERR_INVALID_ARG, "grid dimensions must lie in [1, 2^20]");
    const int64_t bins = (int64_t)grid_rows * grid_cols;
    if (bins > (int64_t(1) << 30)) return fail(MXE_ERR_INVALID_ARG, "more than 2^30 bins");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    hipStream_t s = (hipStream_t)stream;
    if (A->nnz == 0) {
        *h_bits = 0.0;
        if (h_nats) *h_nats = 0.0;
        if (hist) std::fill(hist, hist + bins, (int64_t)0);
        return MXE_OK;
    }
    Scratch hdev, ws, res;
    mxe_status st;
    if ((st = hdev.alloc(4 * (size_t)bins, s))) return st;
    if ((st = ws.alloc(entropy_ws_bytes(bins), s))) return st;
    if ((st = res.alloc(4 * sizeof(double), s))) return st;
    MXE_HIP(launch_block_hist(A->nrows, A->ncols, A->nnz, A->rp, A->col, grid_rows, grid_cols,
                              (uint32_t *)hdev.p, s));
    MXE_HIP(launch_entropy((const uint32_t *)hdev.p, bins, (double *)res.p, ws.p, s));
    double r[4];
    MXE_HIP(hipMemcpyAsync(r, res.p, sizeof r, hipMemcpyDeviceToHost, s));
    std::vector<uint32_t> h32;
    if (hist) {
        h32.resize((size_t)bins);
        MXE_HIP(hipMemcpyAsync(h32.data(), hdev.p, 4 * (size_t)bins, hipMemcpyDeviceToHost, s));
    }
    MXE_HIP(hipStreamSynchronize(s));
    *h_bits = r[0];
    if (h_nats) *h_nats = r[1];
    if (hist) for (int64_t i = 0; i < bins; ++i) hist[i] = h32[(size_t)i];
    if (r[2] != 1.0) return fail(MXE_ERR_INEXACT, "entropy rounding could not be certified");
    return MXE_OK;
}

mxe_status mxe_entropy_levels(mxe_ctx *ctx, mxe_mat m, int32_t grid_rows, int32_t grid_cols,
                              const int32_t *levels, int32_t nlevels, void *stream,
                              double *h_bits, double *h_nats) {
    if (!ctx || !h_bits || !levels) return fail(MXE_ERR_INVALID_ARG, "ctx, levels or h_bits is NULL");
    if (grid_rows < 1 || grid_cols < 1 || grid_rows > (1 << 20) || grid_cols > (1 << 20))
        return fail(MXE_ERR_INVALID_ARG, "grid dimensions must lie in [1, 2^20]");
    const int64_t bins = (int64_t)grid_rows * grid_cols;
    if (bins > (int64_t(1) << 30)) return fail(MXE_ERR_INVALID_ARG, "more than 2^30 bins");
    if (nlevels < 1 || nlevels > 16) return fail(MXE_ERR_INVALID_ARG, "1..16 levels");
    for (int32_t i = 0; i < nlevels; ++i)
        if (levels[i] < 1 || levels[i] > 64) return fail(MXE_ERR_INVALID_ARG, "levels must lie in [1, 64]");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    const int32_t nreg = entropy_regions_count(grid_rows, grid_cols, levels, nlevels);
    if (A->nnz == 0) {
        std::fill(h_bits, h_bits + nreg, 0.0);
        if (h_nats) std::fill(h_nats, h_nats + nreg, 0.0);
        return MXE_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    Scratch hdev, ws, res;
    mxe_status st;
    if ((st = hdev.alloc(4 * (size_t)bins, s))) return st;
    if ((st = ws.alloc(entropy_regions_ws_bytes(grid_rows, grid_cols, levels, nlevels), s))) return st;
    if ((st = res.alloc(4 * sizeof(double) * (size_t)nreg, s))) return st;
    MXE_HIP(launch_block_hist(A->nrows, A->ncols, A->nnz, A->rp, A->col, grid_rows, grid_cols,
                              (uint32_t *)hdev.p, s));
    MXE_HIP(launch_entropy_regions((const uint32_t *)hdev.p, grid_rows, grid_cols, levels, nlevels,
                                   (double *)res.p, ws.p, s));
    std::vector<double> r(4 * (size_t)nreg);
    MXE_HIP(hipMemcpyAsync(r.data(), res.p, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s));
    MXE_HIP(hipStreamSynchronize(s));
    bool ok = true;
    for (int32_t i = 0; i < nreg; ++i) {
        h_bits[i] = r[4 * (size_t)i];
        if (h_nats) h_nats[i] = r[4 * (size_t)i + 1];
        ok = ok && r[4 * (size_t)i + 2] == 1.0;
    }
    if (!ok) return fail(MXE_ERR_INEXACT, "entropy rounding could not be certified");
    return MXE_OK;
}

static mxe_status check_dense(const Matrix &A, int32_t k, const void *X, int64_t ldx,
                              const void *Y, int64_t ldy) {
    if (k < 1) return fail(MXE_ERR_INVALID_ARG, "k must be >= 1");
    if (ldx < k || ldy < k) return fail(MXE_ERR_INVALID_ARG, "leading dimension < k");
    if ((A.ncols > 0 && !X) || (A.nrows > 0 && !Y)) return fail(MXE_ERR_INVALID_ARG, "NULL X or Y");
    return MXE_OK;
}

mxe_status mxe_spmv(mxe_ctx *ctx, mxe_mat m, int32_t k, const void *X, int64_t ldx, void *Y,
                    int64_t ldy, uint32_t flags, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    if (flags & ~MXE_SPACE_ORIGINAL) return fail(MXE_ERR_INVALID_ARG, "unknown flags");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    mxe_status st = check_dense(*A, k, X, ldx, Y, ldy);
    if (st) return st;
    return spmv_internal(ctx, *A, k, X, ldx, Y, ldy, flags, (hipStream_t)stream);
}

// Y = M X over (min, +) or (or, and), 16 columns per launch: on the matrix's
// column-slab layout when its tuned (+, *) variant is one, else the row-group
// semiring kernel. For a permuted matrix in the original index space X is
// gathered by cperm and Y scattered by rperm around the product, as for (+, *).
static mxe_status semiring_core(mxe_ctx *ctx, Matrix &A, int semiring, int32_t k, const void *X,
                                int64_t ldx, void *Y, int64_t ldy, hipStream_t s) {
    const int eb = elem_bytes_of(A.storage);
    for (int32_t c0 = 0; c0 < k; c0 += 16) {
        const int32_t kc = std::min<int32_t>(16, k - c0);
        const void *Xc = (const char *)X + (size_t)c0 * eb;
        void *Yc = (char *)Y + (size_t)c0 * eb;
        TuneResult r;
        mxe_status st = ensure_variant(ctx, A, kc, s, &r);
        if (st) return st;
        if (slab_family(r.variant)) {               // the layout; the window is (+, *) only
            SpmvArgs a;
            if ((st = prepare_args(ctx, A, r.variant, kc, Xc, ldx, Yc, ldy, s, &a))) return st;
            MXE_HIP(launch_spmv_slab(*a.slab, a.vtype, semiring, a.slab_off, a.slab_idx, a.slab_val,
                                     kc, Xc, ldx, Yc, ldy, nullptr, 0, s));
        } else {
            MXE_HIP(launch_spmv_semiring(make_args(A, kc, Xc, ldx, Yc, ldy), semiring, s));
        }
    }
    return MXE_OK;
}

mxe_status mxe_spmv_semiring(mxe_ctx *ctx, mxe_mat m, int32_t semiring, int32_t k, const void *X,
                             int64_t ldx, void *Y, int64_t ldy, uint32_t flags, void *stream) {
    if (semiring == MXE_SR_PLUS_TIMES) return mxe_spmv(ctx, m, k, X, ldx, Y, ldy, flags, stream);
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    if (semiring != MXE_SR_MIN_PLUS && semiring != MXE_SR_OR_AND)
        return fail(MXE_ERR_INVALID_ARG, "unknown semiring");
    if (flags & ~MXE_SPACE_ORIGINAL) return fail(MXE_ERR_INVALID_ARG, "unknown flags");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    mxe_status st = check_dense(*A, k, X, ldx, Y, ldy);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!(flags & MXE_SPACE_ORIGINAL) || !A->rperm) {
        st = semiring_core(ctx, *A, semiring, k, X, ldx, Y, ldy, s);
        return st ? st : note_use(*A, s);
    }
    const int eb = elem_bytes_of(A->storage);
    Scratch xp, yp;
    if ((st = xp.alloc((size_t)eb * std::max(A->ncols, 1) * k, s))) return st;
    if ((st = yp.alloc((size_t)eb * std::max(A->nrows, 1) * k, s))) return st;
    MXE_HIP(launch_gather_rows(A->ncols, k, A->cperm, X, ldx, xp.p, k, eb, s));
    if ((st = semiring_core(ctx, *A, semiring, k, xp.p, k, yp.p, k, s))) return st;
    MXE_HIP(launch_scatter_rows(A->nrows, k, A->rperm, yp.p, k, Y, ldy, eb, s));
    return note_use(*A, s);
}

mxe_status mxe_gather_x(mxe_ctx *ctx, mxe_mat b, int32_t k, const void *X, int64_t ldx, void *Xp,
                        int64_t ldxp, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto B = find_matrix(ctx, b);
    if (!B) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    if (k < 1 || ldx < k || ldxp < k) return fail(MXE_ERR_INVALID_ARG, "bad k or leading dimension");
    if (B->ncols > 0 && (!X || !Xp)) return fail(MXE_ERR_INVALID_ARG, "NULL X or Xp");
    const int eb = elem_bytes_of(B->storage);
    hipStream_t s = (hipStream_t)stream;
    if (!B->cperm) {
        MXE_HIP(launch_copy_cols(B->ncols, k, X, ldx, Xp, ldxp, eb, s));
        return MXE_OK;
    }
    MXE_HIP(launch_gather_rows(B->ncols, k, B->cperm, X, ldx, Xp, ldxp, eb, s));
    return note_use(*B, s);
}

mxe_status mxe_scatter_y(mxe_ctx *ctx, mxe_mat b, int32_t k, const void *Yp, int64_t ldyp, void *Y,
                         int64_t ldy, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto B = find_matrix(ctx, b);
    if (!B) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    if (k < 1 || ldy < k || ldyp < k) return fail(MXE_ERR_INVALID_ARG, "bad k or leading dimension");
    if (B->nrows > 0 && (!Y || !Yp)) return fail(MXE_ERR_INVALID_ARG, "NULL Y or Yp");
    const int eb = elem_bytes_of(B->storage);
    hipStream_t s = (hipStream_t)stream;
    if (!B->rperm) {
        MXE_HIP(launch_copy_cols(B->nrows, k, Yp, ldyp, Y, ldy, eb, s));
        return MXE_OK;
    }
    MXE_HIP(launch_scatter_rows(B->nrows, k, B->rperm, Yp, ldyp, Y, ldy, eb, s));
    return note_use(*B, s);
}

mxe_status mxe_tune(mxe_ctx *ctx, mxe_mat m, int32_t k, void *stream, int32_t *variant) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    if (k < 1) return fail(MXE_ERR_INVALID_ARG, "k must be >= 1");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    TuneResult r;
    mxe_status st = tune(ctx, *A, std::min(k, 16), (hipStream_t)stream, &r);
    if (st) return st;
    if (variant) *variant = r.variant;
    return MXE_OK;
}

mxe_status mxe_probe_gather(mxe_ctx *ctx, int64_t table_bytes, int64_t gathers, int32_t per_xcd,
                            void *stream, double *gathers_per_s) {
    if (!ctx || !gathers_per_s) return fail(MXE_ERR_INVALID_ARG, "ctx or gathers_per_s is NULL");
    if (table_bytes < 64 || table_bytes > (int64_t(1) << 34) || table_bytes % 64)
        return fail(MXE_ERR_INVALID_ARG, "table_bytes must be a multiple of 64 in [64, 2^34]");
    if (gathers < 1 || gathers > (int64_t(1) << 36)) return fail(MXE_ERR_INVALID_ARG, "gathers out of range");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int32_t grid = ctx->cu_count * 8;
    Scratch ws;
    mxe_status st;
    if ((st = ws.alloc(probe_gather_ws_bytes(table_bytes, grid), s))) return st;
    MXE_HIP(hipMemsetAsync(ws.p, 0, (size_t)table_bytes, s));
    hipEvent_t e0, e1;
    MXE_HIP(hipEventCreate(&e0));
    MXE_HIP(hipEventCreate(&e1));
    hipError_t e = launch_probe_gather(table_bytes, gathers, per_xcd, ws.p, grid, s);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_probe_gather(table_bytes, gathers, per_xcd, ws.p, grid, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "gather probe");
    *gathers_per_s = (double)probe_gathers_issued(gathers, grid) / (ms * 1e-3);
    return MXE_OK;
}

mxe_status mxe_set_variant(mxe_ctx *ctx, mxe_mat m, int32_t k, int32_t variant) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    if (k < 1) return fail(MXE_ERR_INVALID_ARG, "k must be >= 1");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto A = find_matrix(ctx, m);
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    const TuneKey key = tune_key(*A, std::min(k, 16));
    if (variant == 0) {
        ctx->tuned.erase(key);
        return MXE_OK;
    }
    if (variant & ~0xfff) return fail(MXE_ERR_INVALID_ARG, "unknown variant");
    const int family = variant & 0xf00, lanes = variant & 0xff;
    const bool pow2 = lanes >= 1 && lanes <= 64 && (lanes & (lanes - 1)) == 0;
    if ((family == MXE_VAR_GROUP || family == MXE_VAR_FIXED) && !pow2)
        return fail(MXE_ERR_INVALID_ARG, "lanes must be 1..64, a power of two");
    if (family != MXE_VAR_GROUP && family != MXE_VAR_BINNED && family != MXE_VAR_MERGE &&
        family != MXE_VAR_SLAB && family != MXE_VAR_FIXED && family != MXE_VAR_COO &&
        family != MXE_VAR_WINDOW)
        return fail(MXE_ERR_INVALID_ARG, "unknown variant family");
    if (slab_family(variant)) {
        SlabGeom sg;
        const int units = slab_units_of(variant);
        if (units < 1 || units > 64)
            return fail(MXE_ERR_INVALID_ARG, "slab size must be 1..64 x 64 KiB");
        if (!layout_geometry(ctx, *A, kclass_of(k), units, slab_cus_of(ctx, variant), &sg))
            return fail(MXE_ERR_UNSUPPORTED, "column-slab layout does not fit this matrix");
        if (family == MXE_VAR_WINDOW && window_rows(ctx, sg, elem_bytes_of(A->storage)) < 1)
            return fail(MXE_ERR_UNSUPPORTED, "no LDS left for an x window in this layout");
    }
    if (family == MXE_VAR_MERGE && kclass_of(k) > 4)
        return fail(MXE_ERR_UNSUPPORTED, "merge-path variant handles k <= 4");
    TuneResult r{variant, family == MXE_VAR_GROUP ? lanes : 8, true};
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end() && family != MXE_VAR_GROUP) r.group_lanes = it->second.group_lanes;
    ctx->tuned[key] = r;
    return MXE_OK;
}

}  // extern "C"

// ---- batches ------------------------------------------------------------------------

namespace mxe {

// work units of one whole batch item: its slab layout's blocks, or row tiles
static int64_t item_units(const BatchDesc &d) {
    return d.slab_off ? d.slab.blocks : (d.nrows + d.rows_per_tile - 1) / d.rows_per_tile;
}

// Deals the items to the per-XCD queues: largest first (bytes one product
// moves) onto the least loaded queue, so each XCD's share is balanced and an
// item's x stays in its own L2. An item moving more than 1/kBatchQueues of the
// batch's bytes would leave its queue the last to finish whatever the others
// hold, so it is first cut into pieces of consecutive work units, each at most
// 1/(2 kBatchQueues) of the bytes (its x is then fetched once per piece's XCD).
// Each queue lists its pieces in item order, with tile_begin counted within
// the queue.
static void assign_queues(std::vector<BatchDesc> &descs, std::vector<uint64_t> &cost,
                          std::vector<int32_t> &qent, BatchQueues &qs) {
    uint64_t total = 0;
    for (uint64_t c : cost) total += c;
    const size_t items = descs.size();
    for (size_t i = 0; i < items; ++i) {
        const int64_t units = descs[i].units;
        if (units < 2 || cost[i] * kBatchQueues <= total) continue;
        // rounded up, so the pieces number at most count + kBatchExtraPieces
        const uint64_t limit = std::max<uint64_t>(1, (total + kBatchExtraPieces - 1) / kBatchExtraPieces);
        const int64_t pieces = std::min<int64_t>(units, (int64_t)((cost[i] + limit - 1) / limit));
        const BatchDesc whole = descs[i];
        const uint64_t c = cost[i];
        for (int64_t p = 0; p < pieces; ++p) {
            const int64_t u0 = units * p / pieces, u1 = units * (p + 1) / pieces;
            BatchDesc d = whole;
            d.unit0 = (int32_t)u0;
            d.units = (int32_t)(u1 - u0);
            const uint64_t pc = (uint64_t)((double)c * (double)(u1 - u0) / (double)units);
            if (p == 0) {
                descs[i] = d;
                cost[i] = pc;
            } else {
                descs.push_back(d);
                cost.push_back(pc);
            }
        }
    }
    const int32_t n = (int32_t)descs.size();
    std::vector<int32_t> order(n), queue_of(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    uint64_t load[kBatchQueues] = {};
    for (int32_t i : order) {
        const int q = (int)(std::min_element(load, load + kBatchQueues) - load);
        queue_of[i] = q;
        load[q] += cost[i];
    }
    qent.clear();
    for (int q = 0; q < kBatchQueues; ++q) {
        qs.qbegin[q] = (int32_t)qent.size();
        int64_t tiles = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (queue_of[i] != q) continue;
            descs[i].tile_begin = (int32_t)tiles;
            tiles += descs[i].units;
            qent.push_back(i);
        }
        qs.qtiles[q] = (int32_t)tiles;
    }
    qs.qbegin[kBatchQueues] = (int32_t)qent.size();
}

// largest slab (in 64 KiB of x) of a batch layout sized for one XCD, and the
// slab of an item not tuned to the slab kernel: with two workgroups per CU an
// XCD works on parts of two or three items at once, and larger slabs of each
// no longer stay together in its L2
constexpr int kBatchSlabUnits = 8;

// One desc per item (before pieces), each item's work unit chosen by the
// batch itself: the blocks of a column-slab layout whose row blocks are sized
// for one XCD's CUs (the item's x is gathered by one XCD) with the tuned slab
// size up to kBatchSlabUnits, or kBatchSlabUnits for an item tuned to a row
// kernel; a slab-tuned item falls back to its tuned layout, any other to row
// tiles of its tuned GROUP lane count, when that layout does not fit the
// matrix or the HBM budget. An
// item whose variant was forced to a row family (mxe_set_variant) runs as row
// tiles. lds: the dynamic LDS the launch needs (the largest slab block's
// partial y).
// The work unit a batch runs A's k-column products as (see build_batch_descs):
// *r the tuning, *out the column-slab layout (null: row tiles). With `prepare`
// it tunes and builds what is missing (stream s); without it, it only looks
// them up. full: prefer the tuned layout, whose row blocks are sized for the
// whole device, to the one sized for one XCD (for an item that is spread over
// the XCDs: one cut into pieces, or one of a batch of few items).
static mxe_status batch_layout(mxe_ctx *ctx, Matrix &A, int32_t k, int32_t index, hipStream_t s,
                               bool prepare, bool full, TuneResult *r, const Matrix::Slab **out) {
    mxe_status st;
    *out = nullptr;
    if (prepare) {
        if ((st = ensure_variant(ctx, A, k, s, r))) return st;
    } else {
        auto tr = ctx->tuned.find(tune_key(A, k));
        if (tr == ctx->tuned.end())
            return fail(MXE_ERR_UNSUPPORTED, "batch item " + std::to_string(index) +
                                                 " is not tuned for its k yet");
        *r = tr->second;
    }
    const bool slab_tuned = slab_family(r->variant);
    if (!slab_tuned && r->forced) return MXE_OK;                // row tiles
    const int kc = kclass_of(k);
    const int xcd_cus = std::max(1, ctx->cu_count / kBatchQueues);
    const int units = slab_tuned ? slab_units_of(r->variant) : kBatchSlabUnits;
    std::vector<int> cus{xcd_cus};
    if (slab_tuned) {
        cus.push_back(slab_cus_of(ctx, r->variant));
        if (full) std::swap(cus[0], cus[1]);
    }
    const Matrix::Slab *sl = nullptr;
    st = MXE_OK;
    // a layout for one XCD takes slabs of at most kBatchSlabUnits, or the
    // fewest 64 KiB more that keep it within 64 slabs
    const int64_t x_bytes = (int64_t)A.ncols * kc * elem_bytes_of(A.storage);
    const int min_units = (int)std::min<int64_t>(64, (x_bytes + 64 * 65536 - 1) / (64 * 65536));
    for (int c : cus) {
        // the tuned layout keeps its slabs
        const int u = (slab_tuned && c == slab_cus_of(ctx, r->variant))
                          ? units
                          : std::max(std::min(units, kBatchSlabUnits), min_units);
        if (prepare) {
            if ((st = ensure_slab(ctx, A, kc, u, c, s, &sl)) == MXE_OK) break;
            sl = nullptr;
        } else {
            // the layout a preparing call would have picked, if it was built
            auto f = A.slabs.find(std::make_tuple(kc, u, c));
            if (f != A.slabs.end()) {
                sl = &f->second;
                break;
            }
        }
    }
    if (!sl && slab_tuned) {
        if (prepare) return st;
        return fail(MXE_ERR_UNSUPPORTED, "batch item " + std::to_string(index) +
                                             " has no slab layout built yet");
    }
    *out = sl;
    return MXE_OK;
}

mxe_status prepare_batch_layout(mxe_ctx *ctx, Matrix &A, int32_t k, hipStream_t s) {
    TuneResult r;
    const Matrix::Slab *sl;
    return batch_layout(ctx, A, k, 0, s, true, false, &r, &sl);
}

mxe_status batch_item_desc(mxe_ctx *ctx, Matrix &A, const mxe_item &it, int32_t index,
                           hipStream_t s, bool prepare, bool full, BatchDesc *out, size_t *lds) {
    if (it.flags != MXE_SPACE_PERMUTED)
        return fail(MXE_ERR_UNSUPPORTED, "batches take permuted-space vectors only");
    if (it.k > 16) return fail(MXE_ERR_UNSUPPORTED, "batches take k <= 16");
    mxe_status st = check_dense(A, it.k, it.X, it.ldx, it.Y, it.ldy);
    if (st) return st;
    TuneResult r;
    const Matrix::Slab *sl;
    if ((st = batch_layout(ctx, A, it.k, index, s, prepare, full, &r, &sl))) return st;
    BatchDesc d{};
    d.rp = A.rp;
    d.col = A.col;
    d.val = A.val;
    d.X = it.X;
    d.Y = it.Y;
    d.ldx = it.ldx;
    d.ldy = it.ldy;
    d.nrows = A.nrows;
    d.k = it.k;
    d.vtype = vtype_of(A.storage);
    d.kclass = kclass_of(it.k);
    d.lanes = std::max(r.group_lanes, d.kclass);   // set_variant may force fewer
    d.rows_per_tile = (kBatchBlock / d.lanes) * 2;
    if (sl) {
        const int eb = elem_bytes_of(A.storage);
        d.slab = sl->g;
        d.slab_off = sl->off;
        d.slab_idx = sl->idx;
        d.slab_val = sl->val;
        d.vec_x = slab_vec_x(d.kclass, it.k, it.X, it.ldx, eb) ? 1 : 0;
        *lds = std::max(*lds, (size_t)sl->g.rows_per_block * d.kclass * eb);
    }
    d.unit0 = 0;
    d.units = (int32_t)item_units(d);
    d.item = index;
    *out = d;
    return MXE_OK;
}

mxe_status build_batch_descs(mxe_ctx *ctx, int32_t count, const mxe_item *items, hipStream_t s,
                             bool prepare, std::vector<BatchDesc> &descs,
                             std::vector<int32_t> &qent, BatchQueues &qs, size_t *lds, bool full) {
    if (count < 1 || !items) return fail(MXE_ERR_INVALID_ARG, "empty batch");
    descs.clear();
    *lds = 0;
    std::vector<std::shared_ptr<Matrix>> mats;
    std::vector<uint64_t> cost;
    uint64_t total = 0;
    for (int32_t i = 0; i < count; ++i) {
        auto A = find_matrix(ctx, items[i].mat);
        if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle in batch");
        if (items[i].flags != MXE_SPACE_PERMUTED)
            return fail(MXE_ERR_UNSUPPORTED, "batches take permuted-space vectors only");
        if (items[i].k > 16) return fail(MXE_ERR_UNSUPPORTED, "batches take k <= 16");
        mxe_status st = check_dense(*A, items[i].k, items[i].X, items[i].ldx, items[i].Y, items[i].ldy);
        if (st) return st;
        cost.push_back(request_bytes(*A, items[i].k));
        total += cost.back();
        mats.push_back(std::move(A));
    }
    int64_t tiles = 0;
    for (int32_t i = 0; i < count; ++i) {
        // an item that assign_queues will cut into pieces is spread over the
        // XCDs anyway: it runs on the layout sized for the whole device
        const bool spread = full || cost[i] * kBatchQueues > total;
        BatchDesc d;
        mxe_status st = batch_item_desc(ctx, *mats[i], items[i], i, s, prepare, spread, &d, lds);
        if (st) return st;
        tiles += d.units;
        if (tiles > INT32_MAX) return fail(MXE_ERR_UNSUPPORTED, "too many tiles in batch");
        descs.push_back(d);
    }
    assign_queues(descs, cost, qent, qs);
    return MXE_OK;
}

int batch_common_vtype(const std::vector<BatchDesc> &descs) {
    for (const BatchDesc &d : descs)
        if (d.vtype != descs[0].vtype) return -1;
    return descs.empty() ? -1 : descs[0].vtype;
}

}  // namespace mxe

extern "C" {

mxe_status mxe_spmv_batch(mxe_ctx *ctx, int32_t count, const mxe_item *items, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<BatchDesc> descs;
    std::vector<int32_t> qent;
    BatchQueues qs{};
    size_t lds = 0;
    mxe_status st = build_batch_descs(ctx, count, items, s, true, descs, qent, qs, &lds);
    if (st) return st;
    const int vt = batch_common_vtype(descs);
    const int32_t grid = batch_grid_size(vt, lds);
    if (grid < 1) return fail(MXE_ERR_DEVICE, "batch kernel occupancy query failed");
    Scratch dd, ctr;
    if ((st = dd.alloc(sizeof(BatchDesc) * descs.size(), s))) return st;
    if ((st = ctr.alloc(sizeof(int32_t) * (kBatchQueues + qent.size()), s))) return st;
    int32_t *counters = (int32_t *)ctr.p;
    MXE_HIP(hipStreamSynchronize(s));     // pool blocks ready before the blocking copies
    MXE_HIP(hipMemcpy(dd.p, descs.data(), sizeof(BatchDesc) * descs.size(), hipMemcpyHostToDevice));
    MXE_HIP(hipMemcpy(counters + kBatchQueues, qent.data(), sizeof(int32_t) * qent.size(),
                      hipMemcpyHostToDevice));
    MXE_HIP(launch_batch_reset(counters, s));
    MXE_HIP(launch_spmv_batch((const BatchDesc *)dd.p, counters + kBatchQueues, qs, counters, grid,
                              lds, vt, s));
    for (int32_t i = 0; i < count; ++i)
        if ((st = note_use(*find_matrix(ctx, items[i].mat), s))) return st;
    return MXE_OK;
}

mxe_status mxe_batch_create(mxe_ctx *ctx, int32_t count, const mxe_item *items, mxe_plan *out) {
    if (!ctx || !out) return fail(MXE_ERR_INVALID_ARG, "ctx or out is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto plan = std::make_unique<Plan>();
    mxe_status st = build_batch_descs(ctx, count, items, nullptr, true, plan->descs, plan->qent,
                                      plan->queues, &plan->lds);
    if (st) return st;
    plan->vtype = batch_common_vtype(plan->descs);
    plan->grid = batch_grid_size(plan->vtype, plan->lds);
    if (plan->grid < 1) return fail(MXE_ERR_DEVICE, "batch kernel occupancy query failed");
    plan->items.assign(items, items + count);
    for (int32_t i = 0; i < count; ++i) plan->mats.push_back(find_matrix(ctx, items[i].mat));
    MXE_HIP(hipEventCreateWithFlags(&plan->done, hipEventDisableTiming));
    MXE_HIP(hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming));
    MXE_HIP(hipHostMalloc((void **)&plan->staging, sizeof(BatchDesc) * plan->descs.size(),
                          hipHostMallocDefault));
    MXE_HIP(hipMalloc(&plan->descs_dev, sizeof(BatchDesc) * plan->descs.size()));
    MXE_HIP(hipMalloc(&plan->counters, sizeof(int32_t) * (kBatchQueues + plan->qent.size())));
    MXE_HIP(hipMemcpy(plan->descs_dev, plan->descs.data(), sizeof(BatchDesc) * plan->descs.size(),
                      hipMemcpyHostToDevice));
    MXE_HIP(hipMemcpy(plan->counters + kBatchQueues, plan->qent.data(),
                      sizeof(int32_t) * plan->qent.size(), hipMemcpyHostToDevice));
    MXE_HIP(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = plan->capture_stream;
    MXE_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = launch_batch_reset(plan->counters, cs);
    hipError_t e2 = launch_spmv_batch(plan->descs_dev, plan->counters + kBatchQueues, plan->queues,
                                      plan->counters, plan->grid, plan->lds, plan->vtype, cs);
    hipError_t e3 = hipStreamEndCapture(cs, &plan->graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)   // ~Plan frees what was made
        return hip_fail(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3, "batch graph capture");
    MXE_HIP(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    const int64_t id = ctx->next_id++;
    ctx->plans[id] = std::move(plan);
    *out = id;
    return MXE_OK;
}

mxe_status mxe_batch_launch(mxe_ctx *ctx, mxe_plan h, const mxe_item *items, void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto it = ctx->plans.find(h);
    if (it == ctx->plans.end()) return fail(MXE_ERR_NOT_FOUND, "unknown plan handle");
    Plan &p = *it->second;
    hipStream_t s = (hipStream_t)stream;
    if (items) {
        for (size_t i = 0; i < p.items.size(); ++i) {
            const mxe_item &a = items[i], &b = p.items[i];
            if (a.mat != b.mat || a.k != b.k || a.flags != b.flags)
                return fail(MXE_ERR_INVALID_ARG, "batch items differ from the plan's matrices or k");
            // the plan's own reference: valid even after the handle was released
            mxe_status st = check_dense(*p.mats[i], a.k, a.X, a.ldx, a.Y, a.ldy);
            if (st) return st;
        }
        bool changed = false;
        for (BatchDesc &d : p.descs) {                  // every piece of every item
            const mxe_item &a = items[d.item];
            if (d.X != a.X || d.Y != a.Y || d.ldx != a.ldx || d.ldy != a.ldy) {
                d.X = a.X;
                d.Y = a.Y;
                d.ldx = a.ldx;
                d.ldy = a.ldy;
                if (d.slab_off)
                    d.vec_x = slab_vec_x(d.kclass, d.k, d.X, d.ldx, d.vtype == VAL_F64 ? 8 : 4) ? 1 : 0;
                changed = true;
            }
        }
        for (size_t i = 0; i < p.items.size(); ++i) p.items[i] = items[i];
        if (changed) {
            // the pinned staging copy is free once the previous rewrite ran;
            // the rewrite itself waits on the device for the previous replay
            MXE_HIP(hipEventSynchronize(p.staged));
            std::memcpy(p.staging, p.descs.data(), sizeof(BatchDesc) * p.descs.size());
            MXE_HIP(hipStreamWaitEvent(s, p.done, 0));
            MXE_HIP(hipMemcpyAsync(p.descs_dev, p.staging, sizeof(BatchDesc) * p.descs.size(),
                                   hipMemcpyHostToDevice, s));
            MXE_HIP(hipEventRecord(p.staged, s));
        }
    }
    // the previous replay (on any stream) shares the work counters: finish it first
    MXE_HIP(hipStreamWaitEvent(s, p.done, 0));
    MXE_HIP(hipGraphLaunch(p.exec, s));
    MXE_HIP(hipEventRecord(p.done, s));
    return MXE_OK;
}

mxe_status mxe_batch_destroy(mxe_ctx *ctx, mxe_plan h) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    auto it = ctx->plans.find(h);
    if (it == ctx->plans.end()) return fail(MXE_ERR_NOT_FOUND, "unknown plan handle");
    ctx->plans.erase(it);                           // ~Plan waits for the last replay
    return MXE_OK;
}

// ---- serving (loop in serve.cpp) -------------------------------------------------------

mxe_status mxe_serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg) {
    if (!ctx || !cfg) return fail(MXE_ERR_INVALID_ARG, "ctx or cfg is NULL");
    return serve_start(ctx, cfg);
}
mxe_status mxe_submit(mxe_ctx *ctx, const mxe_item *req, mxe_ticket *out) {
    if (!ctx || !req || !out) return fail(MXE_ERR_INVALID_ARG, "ctx, req or out is NULL");
    return serve_submit(ctx, req, out);
}
mxe_status mxe_wait(mxe_ctx *ctx, mxe_ticket t, int64_t timeout_us, double *latency_us) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    return serve_wait(ctx, t, timeout_us, latency_us);
}
mxe_status mxe_serve_stop(mxe_ctx *ctx) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    return serve_stop(ctx);
}

}  // extern "C"
