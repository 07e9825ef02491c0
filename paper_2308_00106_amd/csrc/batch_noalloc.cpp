// Allocation-free batches: mxe_spmv_batch for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The persistent batch kernel needs a little device memory besides its
// inputs and outputs: the descriptor table of the batch's pieces, the per-XCD
// queue entries and the queue counters. mxe_spmv_batch takes them from the
// stream-ordered pool; here they live in `scratch`, a static device array of
// fixed size. Every GPU holds its own copy of it until the process ends, at
// its own address, which noalloc_init looks up once per device
// (hipGetSymbolAddress) when a context is created on it. Host code only ever
// uses that address, never the array's name (in host code the name is a
// host-side stand-in, not device memory).
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

namespace mxe {

namespace {

constexpr size_t kCounterBytes = 256;                     // kBatchQueues queue counters
constexpr size_t kMaxPieces = MXE_NOALLOC_MAX_ITEMS + kBatchExtraPieces;
constexpr size_t kQentBytes = (sizeof(int32_t) * kMaxPieces + 255) / 256 * 256;
constexpr size_t kDescBytes = (sizeof(BatchDesc) * kMaxPieces + 255) / 256 * 256;
static_assert(sizeof(int32_t) * kBatchQueues <= kCounterBytes, "queue counters");
static_assert(kCounterBytes + kQentBytes + kDescBytes <= MXE_NOALLOC_SCRATCH_BYTES,
              "the scratch array holds what the header states");

static __device__ __align__(256) unsigned char scratch[MXE_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<void *> g_ptr;                                // per device: scratch's device address

void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    return device >= 0 && (size_t)device < g_ptr.size() ? g_ptr[device] : nullptr;
}

}  // namespace

mxe_status noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0) return fail(MXE_ERR_INVALID_ARG, "device index out of range");
    if ((size_t)device < g_ptr.size() && g_ptr[device]) return MXE_OK;
    DeviceGuard g(device);
    void *p = nullptr;
    MXE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MXE_ERR_DEVICE, "no device address for the batch scratch array");
    if (g_ptr.size() <= (size_t)device) g_ptr.resize(device + 1, nullptr);
    g_ptr[device] = p;
    return MXE_OK;
}

}  // namespace mxe

using namespace mxe;

extern "C" mxe_status mxe_spmv_batch_noalloc(mxe_ctx *ctx, int32_t count, const mxe_item *items,
                                             void *stream) {
    if (!ctx) return fail(MXE_ERR_INVALID_ARG, "ctx is NULL");
    if (count < 1 || !items) return fail(MXE_ERR_INVALID_ARG, "empty batch");
    if (count > MXE_NOALLOC_MAX_ITEMS)
        return fail(MXE_ERR_INVALID_ARG, "an allocation-free batch holds at most " +
                                             std::to_string(MXE_NOALLOC_MAX_ITEMS) + " items");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    char *base = (char *)scratch_of(ctx->device);
    if (!base) return fail(MXE_ERR_DEVICE, "batch scratch array not set up on this device");
    hipStream_t s = (hipStream_t)stream;
    std::vector<BatchDesc> descs;
    std::vector<int32_t> qent;
    BatchQueues qs{};
    size_t lds = 0;
    mxe_status st = build_batch_descs(ctx, count, items, s, false, descs, qent, qs, &lds);
    if (st) return st;
    if (qent.size() * sizeof(int32_t) > kQentBytes || descs.size() * sizeof(BatchDesc) > kDescBytes)
        return fail(MXE_ERR_INVALID_ARG, "batch exceeds the scratch array");
    const int vt = batch_common_vtype(descs);
    const int32_t grid = batch_grid_size(vt, lds);
    if (grid < 1) return fail(MXE_ERR_DEVICE, "batch kernel occupancy query failed");
    int32_t *counters = (int32_t *)base;
    int32_t *qent_dev = (int32_t *)(base + kCounterBytes);
    BatchDesc *descs_dev = (BatchDesc *)(base + kCounterBytes + kQentBytes);
    // stream-ordered after any earlier use of the array on s; the sources are
    // pageable host memory, which the copies have consumed when they return
    MXE_HIP(hipMemcpyAsync(descs_dev, descs.data(), sizeof(BatchDesc) * descs.size(),
                           hipMemcpyHostToDevice, s));
    MXE_HIP(hipMemcpyAsync(qent_dev, qent.data(), sizeof(int32_t) * qent.size(),
                           hipMemcpyHostToDevice, s));
    MXE_HIP(launch_batch_reset(counters, s));                // the counters start at zero
    MXE_HIP(launch_spmv_batch(descs_dev, qent_dev, qs, counters, grid, lds, vt, s));
    for (int32_t i = 0; i < count; ++i)
        if ((st = note_use(*find_matrix(ctx, items[i].mat), s))) return st;
    return MXE_OK;
}
