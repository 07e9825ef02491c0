// Host-side runtime state behind the C ABI (context, matrices, plans,
// serving loop). Shared by api.cpp and serve.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/mxe.h"
#include "internal.h"

namespace mxe {

void set_error(const std::string &msg);
mxe_status fail(mxe_status s, const std::string &msg);
mxe_status hip_fail(hipError_t e, const char *what);

#define MXE_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::mxe::hip_fail(_e, #call);        \
    } while (0)

// Makes `dev` current for a scope and restores the previous device after it.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Matrix {
    int64_t id = 0;
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    mxe_dtype storage = MXE_F64;
    int32_t *rp = nullptr, *col = nullptr;
    void *val = nullptr;
    // permutation (device, new-to-old and old-to-new); null when not permuted
    int32_t *rperm = nullptr, *cperm = nullptr, *rinv = nullptr, *cinv = nullptr;
    std::shared_ptr<Matrix> parent;
    uint64_t seed = 0;
    uint32_t mode = 0;
    uint64_t bytes = 0;                 // HBM held
    // lazily built
    int32_t max_row = -1;
    int32_t *bin_list = nullptr;
    int32_t *bin_off_dev = nullptr;
    int32_t bin_off[kNumBins + 1] = {};
    bool bins_ready = false;
    void *merge_coords = nullptr;       // merge-path slice starts (an entry of allocs)
    int32_t *coo_row = nullptr;         // COO row index per entry (an entry of allocs)
    struct Slab {
        SlabGeom g;
        int32_t *off = nullptr;
        uint32_t *idx = nullptr;
        void *val = nullptr;
        // MXE_VAR_WINDOW on this layout (built on first use): per-block window
        // starts and the window's rows of x
        int32_t *wstart = nullptr;
        int32_t win = 0;
    };
    // (k class, slab size in 64 KiB, CUs the geometry is sized for) -> layout
    std::map<std::tuple<int, int, int>, Slab> slabs;
    std::atomic<int> busy{0};           // serving requests queued or running
    std::vector<void *> allocs;         // device allocations to free
    // per stream, an event recorded after the last work queued there on this
    // matrix: freeing waits for these, never for the whole device
    struct Use {
        hipStream_t s;
        hipEvent_t ev;
    };
    std::vector<Use> uses;
};

struct TuneKey {
    int32_t nrows, ncols;
    int64_t nnz;
    int32_t storage, kclass;
    uint64_t seed;
    uint32_t mode;
    int64_t root;                       // id of the unpermuted ancestor
    bool operator<(const TuneKey &o) const {
        return std::tie(nrows, ncols, nnz, storage, kclass, seed, mode, root) <
               std::tie(o.nrows, o.ncols, o.nnz, o.storage, o.kclass, o.seed, o.mode, o.root);
    }
};
struct TuneResult {
    int variant;
    int group_lanes;
    bool forced = false;                // set by mxe_set_variant, not by the tuner
};

struct Plan {
    std::vector<mxe_item> items;
    std::vector<std::shared_ptr<Matrix>> mats;   // kept alive while the plan exists
    std::vector<BatchDesc> descs;
    BatchDesc *descs_dev = nullptr;
    std::vector<int32_t> qent;          // per-XCD queue entries (desc indices)
    BatchQueues queues{};
    int32_t *counters = nullptr;        // device: kBatchQueues counters, then qent
    size_t lds = 0;                     // dynamic LDS of the launch
    int vtype = -1;                     // ValType shared by the items, or -1
    int32_t grid = 0;                   // resident workgroups of the batch kernel
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    // replays of one plan run one after another, whatever their streams:
    // each waits for `done`, recorded after the previous replay (and before
    // that, the descriptor table's rewrite from the pinned `staging` copy,
    // whose own completion `staged` marks)
    hipEvent_t done = nullptr, staged = nullptr;
    BatchDesc *staging = nullptr;

    Plan() = default;
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    // Frees what the plan holds, whatever step of its creation it reached,
    // after its last replay. The caller has the plan's device current; the
    // matrix references go after the graph (members are destroyed after the body).
    ~Plan() {
        if (done) (void)hipEventSynchronize(done);
        if (staged) (void)hipEventSynchronize(staged);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (descs_dev) (void)hipFree(descs_dev);
        if (counters) (void)hipFree(counters);
        if (staging) (void)hipHostFree(staging);
        if (done) (void)hipEventDestroy(done);
        if (staged) (void)hipEventDestroy(staged);
    }
};

struct Server;

}  // namespace mxe

struct mxe_ctx {
    int device = 0;
    uint64_t budget = 0;                // 0: no cap
    std::atomic<uint64_t> used{0};      // resident bytes
    std::recursive_mutex mu;            // serializes non-serving calls
    std::map<int64_t, std::shared_ptr<mxe::Matrix>> mats;
    std::map<mxe::TuneKey, mxe::TuneResult> tuned;
    std::map<int64_t, std::unique_ptr<mxe::Plan>> plans;
    int64_t next_id = 1;
    int cu_count = 256;
    size_t lds_per_cu = 0, lds_per_block = 0;   // bytes of LDS per CU / per workgroup
    mxe::Server *server = nullptr;      // owned; created and deleted by the serving loop
};

namespace mxe {

// internal helpers implemented in api.cpp, used by serve.cpp
std::shared_ptr<Matrix> find_matrix(mxe_ctx *ctx, mxe_mat m);
// Records that work on A was queued on s (see Matrix::uses).
mxe_status note_use(Matrix &A, hipStream_t s);
mxe_status spmv_internal(mxe_ctx *ctx, Matrix &A, int32_t k, const void *X, int64_t ldx, void *Y,
                         int64_t ldy, uint32_t flags, hipStream_t s);
mxe_status ensure_variant(mxe_ctx *ctx, Matrix &A, int32_t k, hipStream_t s, TuneResult *out);
int elem_bytes_of(mxe_dtype d);
uint64_t request_bytes(const Matrix &A, int32_t k);

// Batches (api.cpp). One item's descriptor, before it is cut into pieces.
// With `prepare`, tunes the item and builds the column-slab layout it runs on
// when they do not exist yet (stream s); without it, only looks them up
// (allocating nothing on the device) and fails with MXE_ERR_UNSUPPORTED for an
// item that is not tuned yet. *lds grows to the dynamic LDS its block needs.
// full: prefer each item's tuned layout (row blocks sized for the whole
// device) to the one sized for one XCD, for batches of few items.
mxe_status batch_item_desc(mxe_ctx *ctx, Matrix &A, const mxe_item &it, int32_t index,
                           hipStream_t s, bool prepare, bool full, BatchDesc *out, size_t *lds);
// Every item's descriptor (batch_item_desc), big items cut into pieces, and
// the pieces dealt to the per-XCD queues.
mxe_status build_batch_descs(mxe_ctx *ctx, int32_t count, const mxe_item *items, hipStream_t s,
                             bool prepare, std::vector<BatchDesc> &descs,
                             std::vector<int32_t> &qent, BatchQueues &qs, size_t *lds,
                             bool full = false);
// Tunes A for k and builds the layouts a batch item of k columns may run on
// (as batch_item_desc with prepare), without an item.
mxe_status prepare_batch_layout(mxe_ctx *ctx, Matrix &A, int32_t k, hipStream_t s);
// the value type every item shares, or -1 (the persistent kernel then carries every path)
int batch_common_vtype(const std::vector<BatchDesc> &descs);

// Allocation-free batches (batch_noalloc.cpp): looks up this device's copy of
// the library's static scratch array once; called by mxe_create with the
// device current.
mxe_status noalloc_init(int device);

// serving loop (serve.cpp)
mxe_status serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg);
mxe_status serve_submit(mxe_ctx *ctx, const mxe_item *req, mxe_ticket *out);
mxe_status serve_wait(mxe_ctx *ctx, mxe_ticket t, int64_t timeout_us, double *latency_us);
mxe_status serve_stop(mxe_ctx *ctx);
void serve_destroy(mxe_ctx *ctx);

}  // namespace mxe
