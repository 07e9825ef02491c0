// Serving loop: continuous batching of SpMV requests on resident, permuted
// matrices (the reuse case of Sections 1 and 7: permute once, multiply many
// times).
//
// One scheduler thread per context. It admits queued requests while a slot is
// free and the HBM budget covers the resident matrices plus the vectors of
// every request in flight, merges queued requests on the same matrix into one
// multi-right-hand-side product (packed into a staging matrix, so the sparse
// matrix streams once for all of them), issues each launch on whichever of
// several device streams has the least work queued, so launches overlap and
// small requests do not wait behind large ones, and retires requests when their
// completion event fires. Requests arriving while others run are admitted as
// soon as slots and budget free up.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>

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
    uint64_t bytes = 0;                 // HBM held while in flight
};

struct Launch {
    std::vector<std::shared_ptr<Request>> reqs;
    hipEvent_t ev = nullptr;
    uint64_t bytes = 0;
    uint64_t work = 0;                  // bytes the product moves (matrix and vectors)
    int stream = 0;                     // index into Server::streams
};

}  // namespace

struct Server {
    mxe_ctx *ctx = nullptr;
    mxe_serve_config cfg{};
    std::vector<hipStream_t> streams;
    std::vector<uint64_t> stream_work;   // bytes of the products queued on each stream
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

    void run();
    void retire_done();
    bool admit_one(std::unique_lock<std::mutex> &lk);
    mxe_status issue(std::vector<std::shared_ptr<Request>> &group, hipStream_t s);
};

static uint64_t vector_bytes(const Matrix &A, int32_t k) {
    return (uint64_t)k * ((uint64_t)A.ncols + A.nrows) * elem_bytes_of(A.storage);
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
        stream_work[l.stream] -= l.work;
        free_events.push_back(l.ev);
        inflight[i] = std::move(inflight.back());
        inflight.pop_back();
        cv_done.notify_all();
    }
}

mxe_status Server::issue(std::vector<std::shared_ptr<Request>> &group, hipStream_t s) {
    Matrix &A = *group[0]->mat;
    const uint32_t flags = group[0]->item.flags;
    const int eb = elem_bytes_of(A.storage);
    if (group.size() == 1) {
        const mxe_item &it = group[0]->item;
        return spmv_internal(ctx, A, it.k, it.X, it.ldx, it.Y, it.ldy, flags, s);
    }
    int32_t K = 0;
    for (auto &r : group) K += r->item.k;
    void *xp = nullptr, *yp = nullptr;
    MXE_HIP(hipMallocAsync(&xp, (size_t)eb * std::max(A.ncols, 1) * K, s));
    hipError_t e = hipMallocAsync(&yp, (size_t)eb * std::max(A.nrows, 1) * K, s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(xp, s);
        return hip_fail(e, "hipMallocAsync(packed Y)");
    }
    mxe_status st = MXE_OK;
    int32_t c = 0;
    for (auto &r : group) {
        const mxe_item &it = r->item;
        e = launch_copy_cols(A.ncols, it.k, it.X, it.ldx, (char *)xp + (size_t)c * eb, K, eb, s);
        if (e != hipSuccess) st = hip_fail(e, "pack X");
        c += it.k;
    }
    if (st == MXE_OK) st = spmv_internal(ctx, A, K, xp, K, yp, K, flags, s);
    c = 0;
    for (auto &r : group) {
        const mxe_item &it = r->item;
        if (st == MXE_OK) {
            e = launch_copy_cols(A.nrows, it.k, (char *)yp + (size_t)c * eb, K, it.Y, it.ldy, eb, s);
            if (e != hipSuccess) st = hip_fail(e, "unpack Y");
        }
        c += it.k;
    }
    (void)hipFreeAsync(xp, s);
    (void)hipFreeAsync(yp, s);
    return st;
}

// Admits the head of the queue (plus mergeable requests) if a slot and the
// budget allow it. Returns false when nothing more can be admitted now.
bool Server::admit_one(std::unique_lock<std::mutex> &lk) {
    if (queue.empty() || inflight_reqs >= cfg.max_inflight) return false;
    std::shared_ptr<Request> head = queue.front();
    std::vector<std::shared_ptr<Request>> group{head};
    int32_t K = head->item.k;
    if (cfg.max_merge_k > 1 && K < cfg.max_merge_k) {
        for (size_t i = 1; i < queue.size() && inflight_reqs + (int)group.size() < cfg.max_inflight;
             ++i) {
            auto &r = queue[i];
            if (r->mat.get() == head->mat.get() && r->item.flags == head->item.flags &&
                K + r->item.k <= cfg.max_merge_k) {
                group.push_back(r);
                K += r->item.k;
            }
        }
    }
    uint64_t bytes = vector_bytes(*head->mat, K);
    if (group.size() > 1) bytes *= 2;                  // packed staging copies
    if (ctx->budget) {
        const uint64_t resident = ctx->used.load();
        if (resident + inflight_bytes + bytes > ctx->budget) {
            if (!inflight.empty()) return false;       // wait for memory to free up
            // nothing runs and it still does not fit: it never will
            head->state = 2;
            head->status = MXE_ERR_BUDGET;
            head->error = "request does not fit the HBM budget";
            head->t_done = Clock::now();
            head->mat->busy--;
            queue.pop_front();
            cv_done.notify_all();
            return true;
        }
    }
    for (auto &r : group)
        for (auto it = queue.begin(); it != queue.end(); ++it)
            if (*it == r) {
                queue.erase(it);
                break;
            }
    // the stream with the least work queued, so a small request does not
    // wait behind a large one while another stream is idle
    const int si = (int)(std::min_element(stream_work.begin(), stream_work.end()) - stream_work.begin());
    const uint64_t work = request_bytes(*head->mat, K);
    hipStream_t s = streams[si];
    // reserve the slots and bytes, then issue without holding the queue lock
    // so submitters are not blocked by the device calls
    for (auto &r : group) r->state = 1;
    inflight_reqs += (int)group.size();
    inflight_bytes += bytes;
    hipEvent_t ev = nullptr;
    if (!free_events.empty()) {
        ev = free_events.back();
        free_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    lk.unlock();
    mxe_status st;
    {
        std::lock_guard<std::recursive_mutex> clk(ctx->mu);
        st = issue(group, s);
    }
    const bool recorded = st == MXE_OK && ev && hipEventRecord(ev, s) == hipSuccess;
    lk.lock();
    if (recorded) {
        Launch l;
        l.reqs = group;
        l.ev = ev;
        l.bytes = bytes;
        l.work = work;
        l.stream = si;
        stream_work[si] += work;
        inflight.push_back(std::move(l));
    } else {
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
        while (admit_one(lk)) {
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

mxe_status serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg) {
    if (cfg->streams < 1 || cfg->max_inflight < 1 || cfg->max_merge_k < 1 || cfg->max_merge_k > 16)
        return fail(MXE_ERR_INVALID_ARG, "serve config out of range");
    if (ctx->server) return fail(MXE_ERR_INVALID_ARG, "serving loop already running");
    (void)hipSetDevice(ctx->device);
    auto srv = std::make_unique<Server>();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    for (int i = 0; i < cfg->streams; ++i) {
        hipStream_t s;
        MXE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));   // default priority
        srv->streams.push_back(s);
    }
    srv->stream_work.assign(srv->streams.size(), 0);
    Server *raw = srv.release();
    ctx->server = raw;
    raw->th = std::thread([raw] { raw->run(); });
    return MXE_OK;
}

mxe_status serve_submit(mxe_ctx *ctx, const mxe_item *req, mxe_ticket *out) {
    Server *srv = ctx->server;
    if (!srv) return fail(MXE_ERR_INVALID_ARG, "serving loop not started");
    std::shared_ptr<Matrix> A;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        A = find_matrix(ctx, req->mat);
    }
    if (!A) return fail(MXE_ERR_NOT_FOUND, "unknown matrix handle");
    if (req->k < 1 || req->ldx < req->k || req->ldy < req->k)
        return fail(MXE_ERR_INVALID_ARG, "bad k or leading dimension");
    if ((A->ncols > 0 && !req->X) || (A->nrows > 0 && !req->Y))
        return fail(MXE_ERR_INVALID_ARG, "NULL X or Y");
    if (req->flags & ~MXE_SPACE_ORIGINAL) return fail(MXE_ERR_INVALID_ARG, "unknown flags");
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
    (void)hipSetDevice(ctx->device);
    for (hipStream_t s : srv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : srv->free_events) (void)hipEventDestroy(e);
    ctx->server = nullptr;
    delete srv;
    return MXE_OK;
}

void serve_destroy(mxe_ctx *ctx) {
    if (ctx->server) (void)serve_stop(ctx);
}

}  // namespace mxe
