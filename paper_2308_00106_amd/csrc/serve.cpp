// Serving loop: continuous batching of SpMV requests on resident, permuted
// matrices (the reuse case of Sections 1 and 7: permute once, multiply many
// times).
//
// One scheduler thread per context. It admits queued requests while a slot
// is free and the HBM budget covers the resident matrices plus the vectors of
// every request in flight. Each admission round takes up to max_batch items
// from the queue: an item is one request, or several queued requests on the
// same matrix (permuted index space) merged into one product of up to
// max_merge_k right-hand sides, so the matrix streams once for all of them
// and its gathers fetch wider rows of x instead of being repeated. A lone
// request runs as its own autotuned product; every other round runs its items
// as one launch of the persistent batch kernel (per-XCD work queues), whose
// descriptor table goes to the device from a pinned staging copy that each
// stream owns. A merged item's right-hand sides are packed side by side into
// the stream's staging matrix by one kernel for the whole round, and each of
// its result columns is written straight into its own request's Y (nothing
// is unpacked). Each round goes to the stream with the least work queued, so
// rounds overlap on the device. Requests retire when their round's
// completion event fires; requests that arrive meanwhile are admitted as soon
// as slots and budget free up. Tuning and layout builds happen when a request
// is submitted, in the submitting thread, so the scheduler only issues
// launches.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "runtime.h"

namespace mxe {

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    mxe_ticket id = 0;
    mxe_item item{};
    std::shared_ptr<Matrix> mat;
    Clock::time_point t_submit, t_done;
    int state = 0;                      // 0 queued, 1 running, 2 done
    mxe_status status = MXE_OK;
    std::string error;
};

// One item of a round: one request, or several merged (same matrix).
struct Item {
    std::vector<std::shared_ptr<Request>> reqs;
    int32_t K = 0;                      // right-hand sides in all
};

struct Launch {
    std::vector<std::shared_ptr<Request>> reqs;
    int items = 0;                      // products of the round
    hipEvent_t ev = nullptr;
    uint64_t bytes = 0;                 // in-flight vector bytes (budget)
    uint64_t work = 0;                  // bytes the products move (matrix and vectors)
    int stream = 0;                     // index into Server::streams
    bool table = false;                 // holds its stream's table and staging
};

// A device stream with the table its batch launches read and the staging
// matrix its merged items' right-hand sides are packed into. The table is
// [queue counters | queue entries | descriptors | column outputs | their
// leading dimensions | pack entries] on the device, the same from the queue
// entries on in pinned host memory; a round rewrites them, and the staging
// matrix, only after the previous round that used them on this stream ended.
struct StreamSlot {
    hipStream_t s = nullptr;
    uint64_t work = 0;                  // bytes of the products queued here
    bool table_busy = false;
    char *dev = nullptr;
    char *host = nullptr;
    char *stage = nullptr;
};

constexpr size_t kCounterBytes = 256;
inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }
int32_t kclass_cols(int32_t k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16; }

}  // namespace

struct Server {
    mxe_ctx *ctx = nullptr;
    mxe_serve_config cfg{};
    std::vector<StreamSlot> streams;
    // table geometry (bytes, from the queue entries on)
    size_t cap_descs = 0, cap_cols = 0, cap_pack = 0;
    size_t off_descs = 0, off_ycol = 0, off_ycol_ld = 0, off_pack = 0, table_bytes = 0;
    size_t stage_bytes = 0;             // per stream
    uint64_t reserved = 0;              // staging counted in the context's budget
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<mxe_ticket, std::shared_ptr<Request>> reqs;
    std::vector<Launch> inflight;
    std::vector<hipEvent_t> free_events;
    uint64_t inflight_bytes = 0;
    int inflight_items = 0;             // products on the device (merged requests share one)
    bool stop = false;
    // mirrors of "a request arrived" and stop that the loop can spin on
    // without taking the lock
    std::atomic<uint64_t> arrivals{0};
    std::atomic<bool> stopping{false};
    int64_t next_ticket = 1;
    std::thread th;
    // counters reported at serve_stop when MXE_LOG is set
    int64_t n_rounds = 0, n_items = 0, n_merged = 0, n_single = 0;
    double issue_us = 0.0;

    void run();
    void retire_done();
    bool admit_round(std::unique_lock<std::mutex> &lk);
    mxe_status issue(std::vector<Item> &round, StreamSlot &slot, bool *table);
    mxe_status issue_batch(std::vector<Item> &items, StreamSlot &slot);
    size_t stage_need(const Matrix &A) const;
    void free_slots();
};

static uint64_t vector_bytes(const Matrix &A, int32_t k) {
    return (uint64_t)k * ((uint64_t)A.ncols + A.nrows) * elem_bytes_of(A.storage);
}

static bool batchable(const Request &r) {
    return r.item.flags == MXE_SPACE_PERMUTED && r.item.k <= 16;
}

// staging a merged item on A may take: max_merge_k columns rounded up to their class
size_t Server::stage_need(const Matrix &A) const {
    return round256((size_t)std::max(A.ncols, 1) * kclass_cols(cfg.max_merge_k) *
                    elem_bytes_of(A.storage));
}

void Server::retire_done() {
    for (size_t i = 0; i < inflight.size();) {
        Launch &l = inflight[i];
        hipError_t q = hipEventQuery(l.ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        const auto now = Clock::now();
        for (auto &r : l.reqs) {
            r->state = 2;
            r->t_done = now;
            if (q != hipSuccess) {
                r->status = MXE_ERR_DEVICE;
                r->error = hipGetErrorString(q);
            }
            r->mat->busy--;
        }
        inflight_items -= l.items;
        inflight_bytes -= l.bytes;
        streams[l.stream].work -= l.work;
        if (l.table) streams[l.stream].table_busy = false;
        free_events.push_back(l.ev);
        inflight[i] = std::move(inflight.back());
        inflight.pop_back();
        cv_done.notify_all();
    }
}

// A round's batch items as one persistent launch on slot's stream, after the
// kernel that packs the merged items' right-hand sides into the staging matrix.
mxe_status Server::issue_batch(std::vector<Item> &items, StreamSlot &slot) {
    const int32_t n = (int32_t)items.size();
    std::vector<mxe_item> its(n);
    std::vector<PackCols> pack[2];                      // by element size: 4, 8 bytes
    int32_t max_n[2] = {0, 0};
    std::vector<void *> ycol;
    std::vector<int64_t> ycol_ld;
    std::vector<int32_t> col0(n, -1);                   // first column entry of a merged item
    size_t stage_off = 0;
    for (int32_t i = 0; i < n; ++i) {
        Item &it = items[i];
        if (it.reqs.size() == 1) {
            its[i] = it.reqs[0]->item;
            continue;
        }
        const Matrix &A = *it.reqs[0]->mat;
        const int eb = elem_bytes_of(A.storage);
        const int32_t ld = kclass_cols(it.K);
        char *xs = slot.stage + stage_off;
        stage_off += round256((size_t)std::max(A.ncols, 1) * ld * eb);
        if (stage_off > stage_bytes) return fail(MXE_ERR_UNSUPPORTED, "merged items exceed the staging");
        mxe_item m = it.reqs[0]->item;
        m.k = it.K;
        m.X = xs;
        m.ldx = ld;
        m.Y = xs;                                      // not written: every column has its own output
        m.ldy = ld;
        its[i] = m;
        col0[i] = (int32_t)ycol.size();
        int32_t c = 0;
        for (auto &r : it.reqs) {
            const mxe_item &q = r->item;
            pack[eb == 8].push_back(PackCols{q.X, q.ldx, xs, ld, A.ncols, q.k, c, 0});
            max_n[eb == 8] = std::max(max_n[eb == 8], A.ncols);
            for (int32_t j = 0; j < q.k; ++j) {
                ycol.push_back((char *)q.Y + (size_t)j * eb);
                ycol_ld.push_back(q.ldy);
            }
            c += q.k;
        }
    }
    std::vector<BatchDesc> descs;
    std::vector<int32_t> qent;
    BatchQueues qs{};
    size_t lds = 0;
    // lookups only: submission prepared every item; few items take the
    // tuned layouts, whose blocks are sized for the whole device
    mxe_status st = build_batch_descs(ctx, n, its.data(), slot.s, false, descs, qent, qs, &lds,
                                      n < kBatchQueues);
    if (st) return st;
    const size_t npack = pack[0].size() + pack[1].size();
    if (descs.size() > cap_descs || ycol.size() > cap_cols || npack > cap_pack)
        return fail(MXE_ERR_UNSUPPORTED, "round exceeds the stream's table");
    char *base = slot.dev + kCounterBytes;              // device twin of slot.host
    void **ycol_dev = (void **)(base + off_ycol);
    int64_t *ycol_ld_dev = (int64_t *)(base + off_ycol_ld);
    for (BatchDesc &d : descs) {
        if (col0[d.item] < 0) continue;
        d.ycol = ycol_dev + col0[d.item];
        d.ycol_ld = ycol_ld_dev + col0[d.item];
    }
    const int vt = batch_common_vtype(descs);
    const int32_t grid = batch_grid_size(vt, lds);
    if (grid < 1) return fail(MXE_ERR_DEVICE, "batch kernel occupancy query failed");
    std::memcpy(slot.host, qent.data(), sizeof(int32_t) * qent.size());
    std::memcpy(slot.host + off_descs, descs.data(), sizeof(BatchDesc) * descs.size());
    size_t used = off_descs + sizeof(BatchDesc) * descs.size();
    if (!ycol.empty()) {
        std::memcpy(slot.host + off_ycol, ycol.data(), sizeof(void *) * ycol.size());
        std::memcpy(slot.host + off_ycol_ld, ycol_ld.data(), sizeof(int64_t) * ycol_ld.size());
        used = off_ycol_ld + sizeof(int64_t) * ycol_ld.size();
    }
    if (npack) {
        std::memcpy(slot.host + off_pack, pack[0].data(), sizeof(PackCols) * pack[0].size());
        std::memcpy(slot.host + off_pack + sizeof(PackCols) * pack[0].size(), pack[1].data(),
                    sizeof(PackCols) * pack[1].size());
        used = off_pack + sizeof(PackCols) * npack;
    }
    MXE_HIP(hipMemcpyAsync(base, slot.host, used, hipMemcpyHostToDevice, slot.s));
    const PackCols *pk = (const PackCols *)(base + off_pack);
    MXE_HIP(launch_pack_cols(pk, (int32_t)pack[0].size(), max_n[0], 4, slot.s));
    MXE_HIP(launch_pack_cols(pk + pack[0].size(), (int32_t)pack[1].size(), max_n[1], 8, slot.s));
    int32_t *counters = (int32_t *)slot.dev;
    MXE_HIP(launch_batch_reset(counters, slot.s));
    MXE_HIP(launch_spmv_batch((const BatchDesc *)(base + off_descs), (const int32_t *)base, qs,
                              counters, grid, lds, vt, slot.s));
    for (Item &it : items)
        if ((st = note_use(*it.reqs[0]->mat, slot.s))) return st;
    return MXE_OK;
}

// A round's launches on slot's stream: a lone unmerged request as its own
// product; otherwise the batch items as one persistent launch (the stream's
// table is free: admit_round chose such a stream) and every other request as
// its own product. *table: the round took the table and staging.
mxe_status Server::issue(std::vector<Item> &round, StreamSlot &slot, bool *table) {
    *table = false;
    std::vector<Item> batch;
    std::vector<std::shared_ptr<Request>> single;
    for (Item &it : round) {
        if (it.reqs.size() > 1 || batchable(*it.reqs[0])) batch.push_back(it);
        else single.push_back(it.reqs[0]);
    }
    if (batch.size() == 1 && batch[0].reqs.size() == 1) {
        single.push_back(batch[0].reqs[0]);
        batch.clear();
    }
    if (!batch.empty()) {
        mxe_status st = issue_batch(batch, slot);
        if (st) return st;
        *table = true;
    }
    for (auto &r : single) {
        const mxe_item &it = r->item;
        mxe_status st = spmv_internal(ctx, *r->mat, it.k, it.X, it.ldx, it.Y, it.ldy, it.flags, slot.s);
        if (st) return st;
    }
    return MXE_OK;
}

// Admits the next round if a slot and the budget allow it: up to max_batch
// items from the queue in arrival order (each new item takes one of the
// max_inflight slots), later requests on an item's matrix merged into it
// (without a slot of their own) while its right-hand sides stay within
// max_merge_k and the staging has room. Returns false when nothing more can
// be admitted now.
bool Server::admit_round(std::unique_lock<std::mutex> &lk) {
    if (queue.empty() || inflight_items >= cfg.max_inflight) return false;
    std::vector<Item> round;
    std::vector<size_t> taken;
    uint64_t bytes = 0;
    size_t stage_used = 0;
    const uint64_t resident = ctx->used.load();
    const size_t scan = std::min(queue.size(), (size_t)4 * cfg.max_inflight + 64);
    for (size_t i = 0; i < scan; ++i) {
        const std::shared_ptr<Request> &r = queue[i];
        const uint64_t b = vector_bytes(*r->mat, r->item.k);
        if (ctx->budget && resident + inflight_bytes + bytes + b > ctx->budget) {
            if (round.empty() && inflight.empty()) {
                // nothing runs and it still does not fit: it never will
                r->state = 2;
                r->status = MXE_ERR_BUDGET;
                r->error = "request does not fit the HBM budget";
                r->t_done = Clock::now();
                r->mat->busy--;
                queue.pop_front();
                cv_done.notify_all();
                return true;
            }
            break;                                     // wait for memory to free up
        }
        bool placed = false;
        if (cfg.max_merge_k > 1 && batchable(*r)) {
            for (Item &it : round) {
                const Request &h = *it.reqs[0];
                if (h.mat.get() != r->mat.get() || !batchable(h) ||
                    it.K + r->item.k > cfg.max_merge_k)
                    continue;
                const size_t need = it.reqs.size() == 1 ? stage_need(*r->mat) : 0;
                if (stage_used + need > stage_bytes) continue;
                stage_used += need;
                it.reqs.push_back(r);
                it.K += r->item.k;
                placed = true;
                break;
            }
        }
        if (!placed) {
            if ((int)round.size() >= cfg.max_batch ||
                inflight_items + (int)round.size() >= cfg.max_inflight)
                continue;                              // only merges fit now
            round.push_back(Item{{r}, r->item.k});
        }
        taken.push_back(i);
        bytes += b;
    }
    if (round.empty()) return false;
    const bool needs_table = round.size() > 1 || round[0].reqs.size() > 1;
    // the stream with the least work queued; a round that uses the table
    // takes a stream whose table is free, and waits if none is
    int si = -1;
    for (int i = 0; i < (int)streams.size(); ++i) {
        if (needs_table && streams[i].table_busy) continue;
        if (si < 0 || streams[i].work < streams[si].work) si = i;
    }
    if (si < 0) return false;
    for (size_t j = taken.size(); j-- > 0;) queue.erase(queue.begin() + taken[j]);
    std::vector<std::shared_ptr<Request>> reqs_of_round;
    uint64_t work = 0;
    for (Item &it : round) {
        work += request_bytes(*it.reqs[0]->mat, it.K);
        for (auto &r : it.reqs) {
            r->state = 1;
            reqs_of_round.push_back(r);
        }
    }
    inflight_items += (int)round.size();
    inflight_bytes += bytes;
    StreamSlot &slot = streams[si];                     // only this thread touches the slots
    hipEvent_t ev = nullptr;
    if (!free_events.empty()) {
        ev = free_events.back();
        free_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    // issue without holding the queue lock, so submitters are not blocked by
    // the device calls
    lk.unlock();
    mxe_status st;
    bool table = false;
    const auto t_issue = Clock::now();
    {
        std::lock_guard<std::recursive_mutex> clk(ctx->mu);
        DeviceGuard g(ctx->device);
        st = issue(round, slot, &table);
    }
    issue_us += std::chrono::duration<double, std::micro>(Clock::now() - t_issue).count();
    ++n_rounds;
    n_items += (int64_t)round.size();
    for (Item &it : round) (it.reqs.size() > 1 ? n_merged : n_single) += (int64_t)it.reqs.size();
    if (table) slot.table_busy = true;
    const bool recorded = st == MXE_OK && ev && hipEventRecord(ev, slot.s) == hipSuccess;
    // untracked, what did launch may still read the stream's table and
    // staging: let it end before the next round may rewrite them
    if (!recorded && table) (void)hipStreamSynchronize(slot.s);
    lk.lock();
    if (recorded) {
        Launch l;
        l.reqs = std::move(reqs_of_round);
        l.items = (int)round.size();
        l.ev = ev;
        l.bytes = bytes;
        l.work = work;
        l.stream = si;
        l.table = table;
        slot.work += work;
        inflight.push_back(std::move(l));
    } else {
        if (table) slot.table_busy = false;            // nothing of this round is tracked
        inflight_items -= (int)round.size();
        inflight_bytes -= bytes;
        if (ev) free_events.push_back(ev);
        const auto now = Clock::now();
        for (auto &r : reqs_of_round) {
            r->state = 2;
            r->status = st == MXE_OK ? MXE_ERR_DEVICE : st;
            r->error = "launch failed";
            r->t_done = now;
            r->mat->busy--;
        }
        cv_done.notify_all();
    }
    return true;
}

// how long the loop spins for new requests: while products run, between two
// polls of their completion events; when nothing runs, before it sleeps
constexpr std::chrono::microseconds kBusySpin{2}, kIdleSpin{2000};

void Server::run() {
    (void)hipSetDevice(ctx->device);
    // timed waits of this thread end on time: Linux otherwise lets a
    // normal thread's timers slip by up to 50 us, which would add that
    // much to every request's completion
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        retire_done();
        while (admit_round(lk)) {
        }
        if (stop && queue.empty() && inflight.empty()) break;
        // Spin without the lock until a request arrives, for a few
        // microseconds while products run (then poll their events again) and
        // for up to kIdleSpin when idle before sleeping: a sleeping thread
        // takes tens of microseconds to wake, which a lone request would add
        // to its latency.
        const bool idle = inflight.empty() && queue.empty();
        const uint64_t seen = arrivals.load(std::memory_order_acquire);
        lk.unlock();
        const auto until = Clock::now() + (idle ? kIdleSpin : kBusySpin);
        bool arrived = false;
        while (!(arrived = arrivals.load(std::memory_order_acquire) != seen) &&
               !stopping.load(std::memory_order_acquire) && Clock::now() < until) {
            for (int i = 0; i < 16; ++i) __builtin_ia32_pause();
        }
        lk.lock();
        if (idle && !arrived && queue.empty() && !stop) cv_work.wait(lk);
    }
}

void Server::free_slots() {
    for (StreamSlot &sl : streams) {
        if (sl.s) {
            (void)hipStreamSynchronize(sl.s);
            (void)hipStreamDestroy(sl.s);
        }
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.stage) (void)hipFree(sl.stage);
    }
    streams.clear();
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    free_events.clear();
    ctx->used -= reserved;
    reserved = 0;
}

mxe_status serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg) {
    if (cfg->streams < 1 || cfg->max_inflight < 1 || cfg->max_batch < 1 ||
        cfg->max_batch > MXE_SERVE_MAX_BATCH || cfg->max_merge_k < 1 || cfg->max_merge_k > 16)
        return fail(MXE_ERR_INVALID_ARG, "serve config out of range");
    if (ctx->server) return fail(MXE_ERR_INVALID_ARG, "serving loop already running");
    DeviceGuard g(ctx->device);
    auto srv = std::make_unique<Server>();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    // a round of n items has at most n + kBatchExtraPieces pieces; a merged
    // item has at most 16 columns and 16 requests (one pack entry each)
    srv->cap_descs = (size_t)cfg->max_batch + kBatchExtraPieces;
    srv->cap_cols = (size_t)cfg->max_batch * 16;
    srv->cap_pack = (size_t)cfg->max_batch * 16;
    srv->off_descs = round256(sizeof(int32_t) * srv->cap_descs);
    srv->off_ycol = srv->off_descs + round256(sizeof(BatchDesc) * srv->cap_descs);
    srv->off_ycol_ld = srv->off_ycol + round256(sizeof(void *) * srv->cap_cols);
    srv->off_pack = srv->off_ycol_ld + round256(sizeof(int64_t) * srv->cap_cols);
    srv->table_bytes = srv->off_pack + round256(sizeof(PackCols) * srv->cap_pack);
    // staging per stream: room for two merged items on the widest resident
    // matrix (a round merges no more than fits; more merges wait)
    if (cfg->max_merge_k > 1) {
        size_t widest = 0;
        {
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            for (auto &kv : ctx->mats) widest = std::max(widest, srv->stage_need(*kv.second));
        }
        srv->stage_bytes = std::max<size_t>(2 * widest, size_t(64) << 20);
    }
    const uint64_t total = (uint64_t)srv->stage_bytes * cfg->streams;
    if (total) {
        if (ctx->budget && ctx->used.load() + total > ctx->budget)
            return fail(MXE_ERR_BUDGET, "no HBM budget left for the serving staging");
        ctx->used += total;
        srv->reserved = total;
    }
    for (int i = 0; i < cfg->streams; ++i) {
        StreamSlot sl;
        hipError_t e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);   // default priority
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dev, kCounterBytes + srv->table_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.host, srv->table_bytes, hipHostMallocDefault);
        if (e == hipSuccess && srv->stage_bytes) e = hipMalloc((void **)&sl.stage, srv->stage_bytes);
        srv->streams.push_back(sl);
        if (e != hipSuccess) {
            srv->free_slots();
            return hip_fail(e, "serving stream setup");
        }
    }
    Server *raw = srv.release();
    ctx->server = raw;
    raw->th = std::thread([raw] { raw->run(); });
    return MXE_OK;
}

// What the scheduler will look up for this request: the matrix's tuning for
// each 16-column chunk and, for a permuted-space request, the layouts a batch
// runs it on, for each k class a merge can reach; built here (default
// stream, synchronized) when missing.
static mxe_status prepare_request(mxe_ctx *ctx, const mxe_serve_config &cfg, Matrix &A,
                                  const mxe_item &req) {
    for (int32_t c0 = 0; c0 < req.k; c0 += 16) {
        TuneResult r;
        mxe_status st = ensure_variant(ctx, A, std::min<int32_t>(16, req.k - c0), nullptr, &r);
        if (st) return st;
    }
    if (req.flags != MXE_SPACE_PERMUTED || req.k > 16) return MXE_OK;
    const int32_t top = kclass_cols(std::max(req.k, cfg.max_merge_k));
    for (int32_t k = kclass_cols(req.k); k <= top; k *= 2) {
        mxe_status st = prepare_batch_layout(ctx, A, k, nullptr);
        if (st) return st;
    }
    return MXE_OK;
}

mxe_status serve_submit(mxe_ctx *ctx, const mxe_item *req, mxe_ticket *out) {
    Server *srv = ctx->server;
    if (!srv) return fail(MXE_ERR_INVALID_ARG, "serving loop not started");
    if (req->k < 1 || req->ldx < req->k || req->ldy < req->k)
        return fail(MXE_ERR_INVALID_ARG, "bad k or leading dimension");
    if (req->flags & ~MXE_SPACE_ORIGINAL) return fail(MXE_ERR_INVALID_ARG, "unknown flags");
    std::shared_ptr<Matrix> A;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        A = find_matrix(ctx, req->mat);
        if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
        if ((A->ncols > 0 && !req->X) || (A->nrows > 0 && !req->Y))
            return fail(MXE_ERR_INVALID_ARG, "NULL X or Y");
        DeviceGuard g(ctx->device);
        mxe_status st = prepare_request(ctx, srv->cfg, *A, *req);
        if (st) return st;
    }
    auto r = std::make_shared<Request>();
    r->item = *req;
    r->mat = A;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(MXE_ERR_INVALID_ARG, "serving loop is stopping");
        r->id = srv->next_ticket++;
        A->busy++;
        srv->reqs[r->id] = r;
        srv->queue.push_back(r);
        srv->arrivals.fetch_add(1, std::memory_order_release);
    }
    srv->cv_work.notify_one();
    *out = r->id;
    return MXE_OK;
}

mxe_status serve_wait(mxe_ctx *ctx, mxe_ticket t, int64_t timeout_us, double *latency_us) {
    Server *srv = ctx->server;
    if (!srv) return fail(MXE_ERR_INVALID_ARG, "serving loop not started");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(t);
    if (it == srv->reqs.end()) return fail(MXE_ERR_NOT_FOUND, "unknown ticket");
    std::shared_ptr<Request> r = it->second;
    auto done = [&] { return r->state == 2; };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return fail(MXE_ERR_TIMEOUT, "request still running");
    }
    srv->reqs.erase(r->id);
    if (latency_us)
        *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    if (r->status != MXE_OK) return fail(r->status, r->error);
    return MXE_OK;
}

mxe_status serve_stop(mxe_ctx *ctx) {
    Server *srv = ctx->server;
    if (!srv) return fail(MXE_ERR_INVALID_ARG, "serving loop not started");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->stopping.store(true, std::memory_order_release);
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    if (getenv("MXE_LOG") && srv->n_rounds)
        fprintf(stderr,
                "[mxe] serving: %lld rounds, %lld items, %lld requests merged, %lld alone, "
                "%.1f us host issue per round\n",
                (long long)srv->n_rounds, (long long)srv->n_items, (long long)srv->n_merged,
                (long long)srv->n_single, srv->issue_us / srv->n_rounds);
    DeviceGuard g(ctx->device);
    srv->free_slots();
    ctx->server = nullptr;
    delete srv;
    return MXE_OK;
}

void serve_destroy(mxe_ctx *ctx) {
    if (ctx->server) (void)serve_stop(ctx);
}

}  // namespace mxe
