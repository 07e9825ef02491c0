// Serving loop: continuous batching of SpMV requests on resident, permuted
// matrices (the reuse case of Sections 1 and 7: permute once, multiply many
// times).
//
// One scheduler thread per context. It admits queued requests in arrival
// order while a slot is free and the HBM budget covers the resident matrices
// plus the vectors of every request in flight. Each admission round takes up
// to max_batch queued requests; its permuted-space requests with k <= 16 run
// as the items of one launch of the persistent batch kernel (per-XCD work
// queues, each request its own item: nothing is packed, merged or copied),
// whose descriptor table goes to the device from a pinned staging copy that
// each stream owns; a lone request, and requests the batch kernel does not
// take, run as their own autotuned products. Each round goes to the stream
// with the least work queued, so rounds overlap on the device and a small
// request does not wait behind a large one while another stream is idle.
// Requests retire when their round's completion event fires; requests that
// arrive meanwhile are admitted as soon as slots and budget free up. Tuning
// and layout builds happen when a request is submitted, in the submitting
// thread, so the scheduler only issues launches.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
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

struct Launch {
    std::vector<std::shared_ptr<Request>> reqs;
    hipEvent_t ev = nullptr;
    uint64_t bytes = 0;                 // in-flight vector bytes (budget)
    uint64_t work = 0;                  // bytes the products move (matrix and vectors)
    int stream = 0;                     // index into Server::streams
    bool table = false;                 // holds its stream's descriptor table
};

// A device stream and the descriptor table of the batch launches issued on
// it: [queue counters | queue entries | descriptors] on the device and the
// same [entries | descriptors] in pinned host memory, which the next launch
// rewrites only after the previous one on this stream has finished.
struct StreamSlot {
    hipStream_t s = nullptr;
    uint64_t work = 0;                  // bytes of the products queued here
    bool table_busy = false;
    char *dev = nullptr;
    char *host = nullptr;
};

constexpr size_t kCounterBytes = 256;
inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

struct Server {
    mxe_ctx *ctx = nullptr;
    mxe_serve_config cfg{};
    std::vector<StreamSlot> streams;
    size_t table_cap = 0;               // descriptors a table holds
    size_t qent_bytes = 0;              // bytes of the queue-entry part
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<mxe_ticket, std::shared_ptr<Request>> reqs;
    std::vector<Launch> inflight;
    std::vector<hipEvent_t> free_events;
    uint64_t inflight_bytes = 0;
    int inflight_reqs = 0;
    bool stop = false;
    int64_t next_ticket = 1;
    std::thread th;
    // counters reported at serve_stop when MXE_LOG is set
    int64_t n_rounds = 0, n_batched = 0, n_single = 0;
    double issue_us = 0.0;

    void run();
    void retire_done();
    bool admit_round(std::unique_lock<std::mutex> &lk);
    mxe_status issue(std::vector<std::shared_ptr<Request>> &group, StreamSlot &slot, bool *table);
    mxe_status issue_batch(std::vector<std::shared_ptr<Request>> &batch, StreamSlot &slot);
    void free_slots();
};

static uint64_t vector_bytes(const Matrix &A, int32_t k) {
    return (uint64_t)k * ((uint64_t)A.ncols + A.nrows) * elem_bytes_of(A.storage);
}

static bool batchable(const Request &r) {
    return r.item.flags == MXE_SPACE_PERMUTED && r.item.k <= 16;
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
            --inflight_reqs;
        }
        inflight_bytes -= l.bytes;
        streams[l.stream].work -= l.work;
        if (l.table) streams[l.stream].table_busy = false;
        free_events.push_back(l.ev);
        inflight[i] = std::move(inflight.back());
        inflight.pop_back();
        cv_done.notify_all();
    }
}

// The batch items of a round as one persistent launch on slot's stream.
mxe_status Server::issue_batch(std::vector<std::shared_ptr<Request>> &batch, StreamSlot &slot) {
    std::vector<mxe_item> items;
    items.reserve(batch.size());
    for (auto &r : batch) items.push_back(r->item);
    std::vector<BatchDesc> descs;
    std::vector<int32_t> qent;
    BatchQueues qs{};
    size_t lds = 0;
    // lookups only: submission prepared every item
    mxe_status st = build_batch_descs(ctx, (int32_t)items.size(), items.data(), slot.s, false, descs,
                                      qent, qs, &lds);
    if (st) return st;
    if (descs.size() > table_cap) return fail(MXE_ERR_UNSUPPORTED, "batch exceeds the stream's table");
    const int vt = batch_common_vtype(descs);
    const int32_t grid = batch_grid_size(vt, lds);
    if (grid < 1) return fail(MXE_ERR_DEVICE, "batch kernel occupancy query failed");
    std::memcpy(slot.host, qent.data(), sizeof(int32_t) * qent.size());
    std::memcpy(slot.host + qent_bytes, descs.data(), sizeof(BatchDesc) * descs.size());
    int32_t *counters = (int32_t *)slot.dev;
    int32_t *qent_dev = (int32_t *)(slot.dev + kCounterBytes);
    const BatchDesc *descs_dev = (const BatchDesc *)(slot.dev + kCounterBytes + qent_bytes);
    MXE_HIP(hipMemcpyAsync(qent_dev, slot.host, qent_bytes + sizeof(BatchDesc) * descs.size(),
                           hipMemcpyHostToDevice, slot.s));
    MXE_HIP(launch_batch_reset(counters, slot.s));
    MXE_HIP(launch_spmv_batch(descs_dev, qent_dev, qs, counters, grid, lds, vt, slot.s));
    for (auto &r : batch)
        if ((st = note_use(*r->mat, slot.s))) return st;
    return MXE_OK;
}

// A round's launches on slot's stream: its batch items (two or more) as one
// persistent launch when the stream's table is free, every other request as
// its own product. *table: the batch launch took the table.
mxe_status Server::issue(std::vector<std::shared_ptr<Request>> &group, StreamSlot &slot, bool *table) {
    std::vector<std::shared_ptr<Request>> batch, single;
    for (auto &r : group) (batchable(*r) ? batch : single).push_back(r);
    *table = false;
    if (batch.size() >= 2 && !slot.table_busy) {
        mxe_status st = issue_batch(batch, slot);
        if (st) return st;
        *table = true;
    } else {
        single.insert(single.end(), batch.begin(), batch.end());
    }
    for (auto &r : single) {
        const mxe_item &it = r->item;
        mxe_status st = spmv_internal(ctx, *r->mat, it.k, it.X, it.ldx, it.Y, it.ldy, it.flags, slot.s);
        if (st) return st;
    }
    return MXE_OK;
}

// Admits the next round (up to max_batch requests from the head of the
// queue) if a slot and the budget allow it. Returns false when nothing more
// can be admitted now.
bool Server::admit_round(std::unique_lock<std::mutex> &lk) {
    if (queue.empty() || inflight_reqs >= cfg.max_inflight) return false;
    std::vector<std::shared_ptr<Request>> group;
    uint64_t bytes = 0;
    const uint64_t resident = ctx->used.load();
    for (size_t i = 0; i < queue.size() && (int)group.size() < cfg.max_batch &&
                       inflight_reqs + (int)group.size() < cfg.max_inflight;
         ++i) {
        const std::shared_ptr<Request> &r = queue[i];
        const uint64_t b = vector_bytes(*r->mat, r->item.k);
        if (ctx->budget && resident + inflight_bytes + bytes + b > ctx->budget) {
            if (group.empty() && inflight.empty()) {
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
        group.push_back(r);
        bytes += b;
    }
    if (group.empty()) return false;
    size_t nbatch = 0;
    for (auto &r : group) nbatch += batchable(*r) ? 1 : 0;
    // the stream with the least work queued; a round with batch items takes
    // one whose table is free, and waits if none is
    int si = -1;
    for (int i = 0; i < (int)streams.size(); ++i) {
        if (nbatch >= 2 && streams[i].table_busy) continue;
        if (si < 0 || streams[i].work < streams[si].work) si = i;
    }
    if (si < 0) return false;
    queue.erase(queue.begin(), queue.begin() + group.size());
    uint64_t work = 0;
    for (auto &r : group) {
        r->state = 1;
        work += request_bytes(*r->mat, r->item.k);
    }
    inflight_reqs += (int)group.size();
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
        st = issue(group, slot, &table);
    }
    issue_us += std::chrono::duration<double, std::micro>(Clock::now() - t_issue).count();
    ++n_rounds;
    (table ? n_batched : n_single) += table ? (int64_t)nbatch : (int64_t)group.size();
    if (table) n_single += (int64_t)(group.size() - nbatch);
    if (table) slot.table_busy = true;
    const bool recorded = st == MXE_OK && ev && hipEventRecord(ev, slot.s) == hipSuccess;
    lk.lock();
    if (recorded) {
        Launch l;
        l.reqs = std::move(group);
        l.ev = ev;
        l.bytes = bytes;
        l.work = work;
        l.stream = si;
        l.table = table;
        slot.work += work;
        inflight.push_back(std::move(l));
    } else {
        if (table) slot.table_busy = false;            // nothing of this round is tracked
        inflight_reqs -= (int)group.size();
        inflight_bytes -= bytes;
        if (ev) free_events.push_back(ev);
        const auto now = Clock::now();
        for (auto &r : group) {
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
        if (inflight.empty() && queue.empty()) {
            cv_work.wait(lk);
        } else {
            // poll device completions; new submissions wake the loop early
            cv_work.wait_for(lk, std::chrono::microseconds(10));
        }
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
    }
    streams.clear();
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    free_events.clear();
}

mxe_status serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg) {
    if (cfg->streams < 1 || cfg->max_inflight < 1 || cfg->max_batch < 1 ||
        cfg->max_batch > MXE_SERVE_MAX_BATCH)
        return fail(MXE_ERR_INVALID_ARG, "serve config out of range");
    if (ctx->server) return fail(MXE_ERR_INVALID_ARG, "serving loop already running");
    DeviceGuard g(ctx->device);
    auto srv = std::make_unique<Server>();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    // a round of n items has at most n + kBatchExtraPieces pieces
    srv->table_cap = (size_t)cfg->max_batch + kBatchExtraPieces;
    srv->qent_bytes = round256(sizeof(int32_t) * srv->table_cap);
    const size_t table = srv->qent_bytes + sizeof(BatchDesc) * srv->table_cap;
    for (int i = 0; i < cfg->streams; ++i) {
        StreamSlot sl;
        hipError_t e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);   // default priority
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dev, kCounterBytes + table);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.host, table, hipHostMallocDefault);
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
// each 16-column chunk and, for a batch item, the layout the batch runs it
// on; built here (default stream, synchronized) when missing.
static mxe_status prepare_request(mxe_ctx *ctx, Matrix &A, const mxe_item &req) {
    for (int32_t c0 = 0; c0 < req.k; c0 += 16) {
        TuneResult r;
        mxe_status st = ensure_variant(ctx, A, std::min<int32_t>(16, req.k - c0), nullptr, &r);
        if (st) return st;
    }
    if (req.flags == MXE_SPACE_PERMUTED && req.k <= 16) {
        BatchDesc d;
        size_t lds = 0;
        return batch_item_desc(ctx, A, req, 0, nullptr, true, &d, &lds);
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
        mxe_status st = prepare_request(ctx, *A, *req);
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
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    if (getenv("MXE_LOG") && srv->n_rounds)
        fprintf(stderr, "[mxe] serving: %lld rounds, %lld requests batched, %lld single, %.1f us host issue per round\n",
                (long long)srv->n_rounds, (long long)srv->n_batched, (long long)srv->n_single,
                srv->issue_us / srv->n_rounds);
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
