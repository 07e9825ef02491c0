// Random-gather rate probe for gfx950: the ceiling that bounds a sparse
// product whose x reads are scattered (the max-entropy case, Section 3).
// Every thread issues 8-byte gathers at indices drawn from a 64-bit LCG, four
// in flight, and keeps one sum, so the only memory traffic is the gathers. With
// `per_xcd` each XCD (workgroups dealt round-robin) gathers only inside its
// own eighth of the table, as the column-slab product does with its slab.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace mxe {

namespace {

constexpr int kProbeBlock = 256;

__device__ inline uint64_t lcg(uint64_t s) { return s * 6364136223846793005ull + 1442695040888963407ull; }

__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const double *__restrict__ table,
                                                              int64_t n, int per_xcd,
                                                              int64_t per_thread, uint64_t seed,
                                                              double *__restrict__ out) {
    const int64_t tid = blockIdx.x * (int64_t)kProbeBlock + threadIdx.x;
    const int64_t span = per_xcd ? n / 8 : n;
    const double *base = per_xcd ? table + (blockIdx.x % 8) * span : table;
    uint64_t s = seed ^ ((uint64_t)tid * 0x9e3779b97f4a7c15ull);
    double acc = 0.0;
    for (int64_t i = 0; i < per_thread; i += 4) {
        int64_t j[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s = lcg(s);
            j[u] = (int64_t)(((s >> 32) * (uint64_t)span) >> 32);   // uniform in [0, span)
        }
        acc += (base[j[0]] + base[j[1]]) + (base[j[2]] + base[j[3]]);
    }
    out[tid] = acc;
}

}  // namespace

size_t probe_gather_ws_bytes(int64_t table_bytes, int32_t grid) {
    return ((size_t)table_bytes + 255) / 256 * 256 + sizeof(double) * (size_t)grid * kProbeBlock;
}

hipError_t launch_probe_gather(int64_t table_bytes, int64_t gathers, int per_xcd, void *ws,
                               int32_t grid, hipStream_t s) {
    double *table = (double *)ws;
    const int64_t n = table_bytes / 8;
    double *out = (double *)((char *)ws + ((size_t)table_bytes + 255) / 256 * 256);
    const int64_t threads = (int64_t)grid * kProbeBlock;
    const int64_t per_thread = std::max<int64_t>(4, (gathers / threads + 3) / 4 * 4);
    hipLaunchKernelGGL(k_probe_gather, dim3(grid), dim3(kProbeBlock), 0, s, (const double *)table,
                       n, per_xcd, per_thread, 0x2545f4914f6cdd1dull, out);
    return hipGetLastError();
}

int64_t probe_gathers_issued(int64_t gathers, int32_t grid) {
    const int64_t threads = (int64_t)grid * kProbeBlock;
    return threads * std::max<int64_t>(4, (gathers / threads + 3) / 4 * 4);
}

}  // namespace mxe
