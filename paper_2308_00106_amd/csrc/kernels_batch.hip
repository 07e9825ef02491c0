// Many matrices in one persistent launch (the reuse setting of Section 1:
// resident, already permuted matrices multiplied again and again).
//
// Each item of a batch is cut into work units: the blocks of a column-slab
// layout, or row tiles. The units sit in one queue per XCD (workgroups are
// dealt to the 8 XCDs round-robin); the host deals items (or, for an item too
// large for one queue, pieces of consecutive units) to the queues, largest
// first onto the least loaded, so an item's x is gathered by one XCD and
// stays in that XCD's L2.
// A workgroup of 1024 threads takes units from its own XCD's queue and, once
// that is empty, from the other queues in turn. Every pull either returns a
// unit or finds a queue exhausted, and each workgroup stops after finding all
// of them exhausted, so the grid always drains.
#include "slab_device.h"
#include "spmv_device.h"

#include <algorithm>

namespace mxe {

static_assert(kBatchBlock == kSlabBlock, "slab units run one layout block per workgroup");

namespace {

// bytes of x per lane each wavefront of a slab unit keeps in flight
constexpr int kBatchInflight = 64;

// Unit u of item d, which the host placed in queue q. A slab unit starts its
// slab rotation at the one tied to q's XCD whichever workgroup runs it, so
// every row's sum is taken in the same order on every launch.
template <typename V, typename T>
__device__ __attribute__((always_inline)) inline void
batch_unit(const BatchDesc &d, int32_t u, int q, unsigned char *smem, int32_t (*soff)[kSlabMax + 1]) {
    // The thread index through an opaque copy per unit: otherwise the
    // compiler hoists the lane arithmetic of every path (each k class, the row
    // tiles) out of the persistent loop and keeps it all live, which costs
    // about 30 registers and half the occupancy.
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    if (d.slab_off) {
        T *yp = reinterpret_cast<T *>(smem);
        const V *sv = as_global((const V *)d.slab_val);
        const T *X = as_global((const T *)d.X);
        T *Y = as_global((T *)d.Y);
        const int32_t *so = as_global(d.slab_off);
        const uint32_t *si = as_global(d.slab_idx);
        void *const *yc = d.ycol ? as_global(d.ycol) : nullptr;
        const int64_t *ycl = d.ycol_ld ? as_global(d.ycol_ld) : nullptr;
#define MXE_BATCH_SLAB(KMV)                                                                        \
    slab_block<V, T, KMV, 0, false, kBatchInflight>(d.slab, u, q, so, si, sv, d.k, X, d.ldx, Y,     \
                                                   d.ldy, d.vec_x, yp, soff, tid, nullptr, 0, 0,  \
                                                   yc, ycl)
        switch (d.slab.kclass) {
        case 1: MXE_BATCH_SLAB(1); break;
        case 2: MXE_BATCH_SLAB(2); break;
        case 4: MXE_BATCH_SLAB(4); break;
        case 8: MXE_BATCH_SLAB(8); break;
        default: MXE_BATCH_SLAB(16); break;
        }
#undef MXE_BATCH_SLAB
    } else {
        const int32_t r0 = u * d.rows_per_tile;
        const int32_t r1 = min(d.nrows, r0 + d.rows_per_tile);
        rows_runtime<V, T, kBatchBlock>(as_global(d.rp), as_global(d.col), as_global((const V *)d.val),
                                       d.k, as_global((const T *)d.X), d.ldx, as_global((T *)d.Y),
                                       d.ldy, d.lanes, d.kclass, r0, r1, tid,
                                       d.ycol ? as_global(d.ycol) : nullptr,
                                       d.ycol_ld ? as_global(d.ycol_ld) : nullptr);
    }
}

// VT is the value type shared by every item, or -1 for a batch that mixes
// them (that instance carries every path and so more code). The FP32-math
// instances are held to two workgroups per CU (8 waves per SIMD): the
// descriptor fields the compiler keeps in scalar registers would otherwise
// take more than the 100 SGPRs that allows, and leave one workgroup per CU.
template <int VT>
__global__ __launch_bounds__(kBatchBlock)
__attribute__((amdgpu_waves_per_eu(VT == VAL_F32 || VT == VAL_BF16 ? 8 : 1)))
void k_spmv_batch(const BatchDesc *__restrict__ descs,
                                                           const int32_t *__restrict__ qent,
                                                           BatchQueues qs, int32_t *counters) {
    // slab units: the block's partial y (16-byte aligned for FP64 and vector LDS access)
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ int32_t soff[kSubBlocks][kSlabMax + 1];
    __shared__ int32_t unit_s;
    const int home = blockIdx.x % kBatchQueues;
    for (int step = 0; step < kBatchQueues;) {
        const int q = (home + step) % kBatchQueues;
        if (threadIdx.x == 0) unit_s = atomicAdd(&counters[q], 1);
        __syncthreads();
        // the same for every lane: readfirstlane lets the item lookup and its
        // fields live in scalar registers
        const int32_t unit = __builtin_amdgcn_readfirstlane(unit_s);
        __syncthreads();                                     // also ends the previous unit's LDS use
        if (unit >= qs.qtiles[q]) {                          // queue exhausted: next one
            ++step;
            continue;
        }
        int32_t lo = qs.qbegin[q], hi = qs.qbegin[q + 1] - 1;   // last item starting <= unit
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (descs[qent[mid]].tile_begin <= unit) lo = mid;
            else hi = mid - 1;
        }
        const BatchDesc &d = descs[qent[lo]];
        const int32_t u = unit - d.tile_begin + d.unit0;
        if constexpr (VT == VAL_F64) {
            batch_unit<double, double>(d, u, q, smem, soff);
        } else if constexpr (VT == VAL_F32) {
            batch_unit<float, float>(d, u, q, smem, soff);
        } else if constexpr (VT == VAL_BF16) {
            batch_unit<uint16_t, float>(d, u, q, smem, soff);
        } else {
            if (d.vtype == VAL_F64) batch_unit<double, double>(d, u, q, smem, soff);
            else if (d.vtype == VAL_F32) batch_unit<float, float>(d, u, q, smem, soff);
            else batch_unit<uint16_t, float>(d, u, q, smem, soff);
        }
    }
}

__global__ void k_batch_reset(int32_t *counters) {
    if (threadIdx.x < kBatchQueues) counters[threadIdx.x] = 0;
}

// workgroups of k_spmv_batch<VT> resident at once on the current device
template <int VT>
int32_t batch_grid(size_t lds) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv_batch<VT>, kBatchBlock, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1)
        return 0;
    return std::max(per_cu * cus, kBatchQueues);
}

}  // namespace

hipError_t launch_batch_reset(int32_t *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kWave), 0, s, counters);
    return hipGetLastError();
}

int32_t batch_grid_size(int vtype, size_t lds_bytes) {
    switch (vtype) {
    case VAL_F64: return batch_grid<VAL_F64>(lds_bytes);
    case VAL_F32: return batch_grid<VAL_F32>(lds_bytes);
    case VAL_BF16: return batch_grid<VAL_BF16>(lds_bytes);
    default: return batch_grid<-1>(lds_bytes);
    }
}

hipError_t launch_spmv_batch(const BatchDesc *descs, const int32_t *qent, const BatchQueues &qs,
                             int32_t *counters, int32_t grid, size_t lds_bytes, int vtype,
                             hipStream_t s) {
    if (qs.qbegin[kBatchQueues] <= 0) return hipSuccess;
    if (grid < 1) return hipErrorInvalidConfiguration;
#define MXE_BATCH_LAUNCH(VTV)                                                                      \
    hipLaunchKernelGGL(k_spmv_batch<VTV>, dim3(grid), dim3(kBatchBlock), lds_bytes, s, descs, qent, \
                       qs, counters)
    switch (vtype) {
    case VAL_F64: MXE_BATCH_LAUNCH(VAL_F64); break;
    case VAL_F32: MXE_BATCH_LAUNCH(VAL_F32); break;
    case VAL_BF16: MXE_BATCH_LAUNCH(VAL_BF16); break;
    default: MXE_BATCH_LAUNCH(-1); break;
    }
#undef MXE_BATCH_LAUNCH
    return hipGetLastError();
}

}  // namespace mxe
