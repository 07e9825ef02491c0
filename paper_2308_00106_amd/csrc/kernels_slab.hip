// Column-slab SpMV for gfx950: the x gathers of a max-entropy matrix made
// L2-resident.
//
// After the random column permutation every row's columns are spread
// uniformly over x (Section 3's aim), so with x larger than one XCD's 4 MB L2
// most gathers miss to the Infinity Cache at a full cache line per 8 useful
// bytes. The paper's custom-hardware answer is a banked x buffer (Section 1);
// the MI355X counterpart is the per-XCD L2.
//
// Layout (built once per matrix and right-hand-side class): columns are cut
// into S slabs whose x slice fits comfortably in one L2; rows are cut into
// workgroup blocks of R rows, each split into 16 wavefront sub-blocks. Entries
// are stored grouped by (block, sub-block, slab), rows ascending inside a
// group, each as one 32-bit word (row in sub-block << cbits | global column)
// plus its value. The product keeps each block's partial y in LDS and walks
// the slabs in a rotation that starts at a slab tied to the workgroup's XCD
// (workgroups are dealt to the 8 XCDs round-robin), so at any moment an XCD's
// workgroups gather from one slab of x that sits in its L2. Because a
// max-entropy matrix gives every (block, slab) tile the same expected nonzero
// count, the workgroups of an XCD stay in step; a barrier after each slab
// keeps the wavefronts of a workgroup together. Each row's sum is taken in a
// fixed order (slabs in rotation order, entries in storage order, a fixed
// segmented scan inside a wavefront), so results are deterministic.
#include "slab_device.h"

#include <algorithm>

namespace mxe {

namespace {

constexpr int kFillBatch = 4;                      // 64-entry chunks loaded together by the build

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int bits_for(int64_t n) {                    // bits to hold 0 .. n-1
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

__device__ inline int32_t slab_of(int32_t col, int32_t width, double inv_w) {
    int32_t q = (int32_t)((double)col * inv_w);
    if ((int64_t)q * width > col) --q;
    else if ((int64_t)(q + 1) * width <= col) ++q;
    return q;
}

// Pass 1: entries per (block, sub-block, slab). Lanes take consecutive
// entries of the wavefront's sub-block (coalesced column loads).
__global__ __launch_bounds__(kSlabBlock) void k_slab_count(SlabGeom g, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           int32_t *__restrict__ cnt) {
    __shared__ int32_t c[kSubBlocks][kSlabMax];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int s = lane; s < g.slabs; s += kWave) c[wave][s] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * g.rows_per_block + (int64_t)wave * g.rows_per_sub;
    const int64_t r1 = std::min<int64_t>(std::min<int64_t>(r0 + g.rows_per_sub,
                                         (int64_t)(blockIdx.x + 1) * g.rows_per_block), g.nrows);
    if (r0 < r1) {
        const double inv_w = 1.0 / g.width;
        const int32_t e1 = rp[r1];
        for (int32_t e = rp[r0] + lane; e < e1; e += kFillBatch * kWave) {
            int32_t cv[kFillBatch];                             // loads of the batch first
#pragma unroll
            for (int j = 0; j < kFillBatch; ++j) cv[j] = e + j * kWave < e1 ? col[e + j * kWave] : -1;
#pragma unroll
            for (int j = 0; j < kFillBatch; ++j)
                if (cv[j] >= 0) atomicAdd(&c[wave][slab_of(cv[j], g.width, inv_w)], 1);
        }
    }
    __syncthreads();
    int32_t *out = cnt + ((int64_t)blockIdx.x * kSubBlocks + wave) * g.slabs;
    for (int s = lane; s < g.slabs; s += kWave) out[s] = c[wave][s];
}

// Pass 2: place every entry. A wavefront walks its sub-block's entries in
// CSR order, 64 at a time, and splits each chunk by slab stably (lanes with
// the same slab found with one ballot per slab-index bit), so entries keep
// CSR order, and hence ascending rows, inside every group. Each entry's row
// comes from a binary search of the sub-block's row_ptr slice kept in LDS.
template <typename V>
__global__ __launch_bounds__(kSlabBlock) void k_slab_fill(SlabGeom g, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col,
                                                          const V *__restrict__ val,
                                                          const int32_t *__restrict__ off,
                                                          uint32_t *__restrict__ idx_out,
                                                          V *__restrict__ val_out) {
    extern __shared__ int32_t rps[];                    // kSubBlocks x (rows_per_sub + 1)
    __shared__ int32_t base[kSubBlocks][kSlabMax];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t *o = off + ((int64_t)blockIdx.x * kSubBlocks + wave) * g.slabs;
    for (int s = lane; s < g.slabs; s += kWave) base[wave][s] = o[s];
    const int64_t r0 = (int64_t)blockIdx.x * g.rows_per_block + (int64_t)wave * g.rows_per_sub;
    const int64_t r1 = std::min<int64_t>(std::min<int64_t>(r0 + g.rows_per_sub,
                                         (int64_t)(blockIdx.x + 1) * g.rows_per_block), g.nrows);
    const int32_t nr = r0 < r1 ? (int32_t)(r1 - r0) : 0;
    int32_t *wrp = rps + wave * (g.rows_per_sub + 1);
    // a wavefront of the last block may own no rows (r0 past the last row):
    // it reads nothing, rp[r0] would lie beyond the array
    if (nr > 0)
        for (int32_t i = lane; i <= nr; i += kWave) wrp[i] = rp[r0 + i];
    __syncthreads();
    if (nr == 0) return;
    const double inv_w = 1.0 / g.width;
    const int32_t e0 = wrp[0], e1 = wrp[nr];
    const uint64_t below = (uint64_t(1) << lane) - 1;
    for (int32_t b0 = e0; b0 < e1; b0 += kFillBatch * kWave) {    // uniform per wavefront
        int32_t cvs[kFillBatch];                                 // the batch's loads first
        V vs[kFillBatch];
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) {
            const int32_t e = b0 + j * kWave + lane;
            cvs[j] = e < e1 ? col[e] : 0;
            vs[j] = e < e1 ? val[e] : V{};
        }
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) {
            const int32_t c0 = b0 + j * kWave;
            if (c0 >= e1) break;                                 // uniform per wavefront
            const int32_t e = c0 + lane;
            const bool valid = e < e1;
            int32_t sl = 0, rloc = 0;
            if (valid) {
                sl = slab_of(cvs[j], g.width, inv_w);
                int32_t lo = 0, hi = nr - 1;                     // last row with wrp[row] <= e
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (wrp[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                rloc = lo;
            }
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 6; ++b) {
                const uint64_t m = __ballot(valid && ((sl >> b) & 1));
                same &= ((sl >> b) & 1) ? m : ~m;
            }
            if (valid) {
                const int32_t pos = base[wave][sl] + __popcll(same & below);
                idx_out[pos] = ((uint32_t)rloc << g.cbits) | (uint32_t)cvs[j];
                val_out[pos] = vs[j];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (valid && (same & below) == 0) base[wave][sl] += __popcll(same);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// The product: one layout block per workgroup (slab_block). WIN: the
// block's x window (wstart[block], win rows) sits in LDS after the partial y.
template <typename V, typename T, int KM, int SR, bool WIN>
__global__ __launch_bounds__(kSlabBlock) void k_spmv_slab(SlabGeom g, const int32_t *__restrict__ off,
                                                          const uint32_t *__restrict__ idx,
                                                          const V *__restrict__ val, int32_t k,
                                                          const T *__restrict__ X, int64_t ldx,
                                                          T *__restrict__ Y, int64_t ldy,
                                                          int vec_x, const int32_t *__restrict__ wstart,
                                                          int32_t win, int prio) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ int32_t soff[kSubBlocks][kSlabMax + 1];
    T *yp = reinterpret_cast<T *>(smem);
    if constexpr (WIN) {
        T *xw = yp + slab_window_offset(g, (int)sizeof(T)) / sizeof(T);
        slab_block<V, T, KM, SR, true>(g, blockIdx.x, blockIdx.x % 8, off, idx, val, k, X, ldx, Y,
                                       ldy, vec_x, yp, soff, threadIdx.x, xw, wstart[blockIdx.x], win,
                                       nullptr, nullptr, prio != 0);
    } else {
        slab_block<V, T, KM, SR>(g, blockIdx.x, blockIdx.x % 8, off, idx, val, k, X, ldx, Y, ldy,
                                 vec_x, yp, soff, threadIdx.x, nullptr, 0, 0, nullptr, nullptr,
                                 prio != 0);
    }
}

// Whether the wavefronts raise their priority around the x gathers (one
// right-hand side): with an x window in LDS, and with one workgroup per CU
// (no more blocks than CUs). Measured on the n = 2M FP64 products; with two
// workgroups per CU and no window it made the product slower.
static int gather_prio(const SlabGeom &g, int32_t win) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return win > 0 || g.blocks <= cus;
}

template <typename V, typename T, int KM, int SR>
hipError_t slab_launch(const SlabGeom &g, const int32_t *off, const uint32_t *idx, const void *val,
                       int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                       const int32_t *wstart, int32_t win, hipStream_t s) {
    size_t lds = (size_t)g.rows_per_block * KM * sizeof(T);
    const int vec_x = slab_vec_x(KM, k, X, ldx, (int)sizeof(T));
    if constexpr (SR == 0) {
        if (win > 0) {
            lds = slab_window_offset(g, (int)sizeof(T)) + (size_t)win * KM * sizeof(T);
            hipLaunchKernelGGL((k_spmv_slab<V, T, KM, SR, true>), dim3(g.blocks), dim3(kSlabBlock),
                               lds, s, g, off, idx, (const V *)val, k, (const T *)X, ldx, (T *)Y,
                               ldy, vec_x, wstart, win, gather_prio(g, win));
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_spmv_slab<V, T, KM, SR, false>), dim3(g.blocks), dim3(kSlabBlock), lds, s,
                       g, off, idx, (const V *)val, k, (const T *)X, ldx, (T *)Y, ldy, vec_x,
                       (const int32_t *)nullptr, 0, gather_prio(g, 0));
    return hipGetLastError();
}

template <typename V, typename T, int SR>
hipError_t slab_by_k(const SlabGeom &g, const int32_t *off, const uint32_t *idx, const void *val,
                     int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                     const int32_t *wstart, int32_t win, hipStream_t s) {
    switch (g.kclass) {
    case 1: return slab_launch<V, T, 1, SR>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case 2: return slab_launch<V, T, 2, SR>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case 4: return slab_launch<V, T, 4, SR>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case 8: return slab_launch<V, T, 8, SR>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case 16: return slab_launch<V, T, 16, SR>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename V, typename T>
hipError_t slab_by_semiring(const SlabGeom &g, int semiring, const int32_t *off, const uint32_t *idx,
                            const void *val, int32_t k, const void *X, int64_t ldx, void *Y,
                            int64_t ldy, const int32_t *wstart, int32_t win, hipStream_t s) {
    switch (semiring) {
    case 0: return slab_by_k<V, T, 0>(g, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case 1: return slab_by_k<V, T, 1>(g, off, idx, val, k, X, ldx, Y, ldy, nullptr, 0, s);
    case 2: return slab_by_k<V, T, 2>(g, off, idx, val, k, X, ldx, Y, ldy, nullptr, 0, s);
    default: return hipErrorInvalidValue;
    }
}

// Window placement: block b's window starts where the most of a sample of
// its stored columns fit into `win` consecutive columns. Up to 1024 entries
// spread evenly over the block's rows are sampled (all of them when fewer),
// sorted in LDS (bitonic network), and each sample i counts the samples in
// [s_i, s_i + win); the first sample with the largest count gives the start,
// moved left when the window would pass the last column.
constexpr int kWinSample = kSlabBlock;
__global__ __launch_bounds__(kSlabBlock) void k_slab_window(SlabGeom g, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            int32_t win, int32_t *__restrict__ wstart) {
    __shared__ int32_t smp[kWinSample];
    __shared__ int64_t best[kSlabBlock / kWave];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * g.rows_per_block;
    const int64_t r1 = std::min<int64_t>(r0 + g.rows_per_block, g.nrows);
    const int64_t e0 = rp[r0], n = rp[r1] - e0;
    const int cnt = (int)std::min<int64_t>(n, kWinSample);
    smp[t] = t < cnt ? col[e0 + (int64_t)t * n / cnt] : INT32_MAX;
    __syncthreads();
    for (int kk = 2; kk <= kWinSample; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const int p = t ^ j;
            if (p > t) {
                const int32_t a = smp[t], b = smp[p];
                if ((a > b) == ((t & kk) == 0)) {
                    smp[t] = b;
                    smp[p] = a;
                }
            }
            __syncthreads();
        }
    // key: count in the high bits, then the lower sample index first
    int64_t key = -1;
    if (t < cnt) {
        const int64_t lim = (int64_t)smp[t] + win;          // first column past the window
        int lo = t, hi = cnt;                                // first sample >= lim
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (smp[mid] < lim) lo = mid + 1;
            else hi = mid;
        }
        key = ((int64_t)(lo - t) << 32) | (uint32_t)(kWinSample - t);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int64_t other = __shfl_xor(key, o);
        key = other > key ? other : key;
    }
    if (t % kWave == 0) best[t / kWave] = key;
    __syncthreads();
    if (t == 0) {
        int64_t b = best[0];
        for (int w = 1; w < kSlabBlock / kWave; ++w) b = best[w] > b ? best[w] : b;
        int64_t start = 0;
        if (b >= 0) start = smp[kWinSample - (int)(b & 0xffffffff)];
        if (start + win > g.ncols) start = std::max<int64_t>(0, (int64_t)g.ncols - win);
        wstart[blockIdx.x] = (int32_t)start;
    }
}

}  // namespace

bool slab_geometry(int32_t nrows, int32_t ncols, int kclass, int vtype, int cu_count,
                   int64_t slab_bytes, int64_t y_lds_bytes, int64_t resident, SlabGeom *g) {
    if (nrows <= 0 || ncols <= 0) return false;
    const int64_t xb = vtype == VAL_F64 ? 8 : 4;
    const int64_t per_col = xb * kclass;
    int64_t slabs = std::max<int64_t>(1, cdiv((int64_t)ncols * per_col, slab_bytes));
    if (slabs > kSlabMax) return false;
    const int64_t width = cdiv(ncols, slabs);
    slabs = cdiv(ncols, width);
    // rows per block: two blocks per CU cover the matrix if the block's
    // partial y fits y_lds_bytes of LDS; else, with resident > 0, the rows are
    // spread evenly over as many whole waves of the `resident` blocks that run
    // at once as that takes, so no wave runs with only a few blocks (with
    // resident 0, blocks of the largest size, for a work queue)
    // (at most 16384 rows: the build's row-start table stays within 64 KiB of LDS)
    const int64_t lds_rows = std::max<int64_t>(
        kSubBlocks, std::min<int64_t>(16384, y_lds_bytes / per_col) / kSubBlocks * kSubBlocks);
    int64_t R = cdiv(nrows, 2 * (int64_t)cu_count);
    if (R > lds_rows) {
        if (resident > 0) {
            const int64_t waves = cdiv(nrows, resident * lds_rows);
            R = cdiv(nrows, waves * resident);
        } else {
            R = lds_rows;
        }
    }
    R = std::max<int64_t>(R, kSubBlocks);
    R = cdiv(R, kSubBlocks) * kSubBlocks;
    // packed words (row in sub-block, global column) stay below 2^31, so they
    // never equal the padding key; smaller blocks free row bits
    const int cbits = bits_for(ncols);
    while (cbits + bits_for(R / kSubBlocks) > 31 && R > kSubBlocks) R = cdiv(R / 2, kSubBlocks) * kSubBlocks;
    const int64_t Rq = R / kSubBlocks;
    if (cbits + bits_for(Rq) > 31) return false;
    g->nrows = nrows;
    g->ncols = ncols;
    g->slabs = (int32_t)slabs;
    g->width = (int32_t)width;
    g->cbits = cbits;
    g->rows_per_block = (int32_t)R;
    g->rows_per_sub = (int32_t)Rq;
    g->blocks = (int32_t)cdiv(nrows, R);
    g->kclass = kclass;
    return true;
}

size_t slab_offsets_count(const SlabGeom &g) { return (size_t)g.blocks * kSubBlocks * g.slabs + 1; }

size_t slab_build_ws_bytes(const SlabGeom &g) { return scan_ws_bytes((int64_t)slab_offsets_count(g)); }

hipError_t launch_slab_build(const SlabGeom &g, const int32_t *rp, const int32_t *col, const void *val,
                             int val_bytes, int32_t *off, uint32_t *idx_out, void *val_out, void *ws,
                             hipStream_t s) {
    const int64_t n = (int64_t)slab_offsets_count(g);
    hipError_t e = launch_fill_i32(off, n, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_slab_count, dim3(g.blocks), dim3(kSlabBlock), 0, s, g, rp, col, off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan(off, off, n, ws, s)) != hipSuccess) return e;
    const size_t rps_lds = sizeof(int32_t) * kSubBlocks * ((size_t)g.rows_per_sub + 1);
    switch (val_bytes) {
    case 8:
        hipLaunchKernelGGL(k_slab_fill<uint64_t>, dim3(g.blocks), dim3(kSlabBlock), rps_lds, s, g, rp, col,
                           (const uint64_t *)val, (const int32_t *)off, idx_out, (uint64_t *)val_out);
        break;
    case 4:
        hipLaunchKernelGGL(k_slab_fill<uint32_t>, dim3(g.blocks), dim3(kSlabBlock), rps_lds, s, g, rp, col,
                           (const uint32_t *)val, (const int32_t *)off, idx_out, (uint32_t *)val_out);
        break;
    case 2:
        hipLaunchKernelGGL(k_slab_fill<uint16_t>, dim3(g.blocks), dim3(kSlabBlock), rps_lds, s, g, rp, col,
                           (const uint16_t *)val, (const int32_t *)off, idx_out, (uint16_t *)val_out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_slab_window(const SlabGeom &g, const int32_t *rp, const int32_t *col, int32_t win,
                              int32_t *wstart, hipStream_t s) {
    if (win < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_slab_window, dim3(g.blocks), dim3(kSlabBlock), 0, s, g, rp, col, win, wstart);
    return hipGetLastError();
}

hipError_t launch_spmv_slab(const SlabGeom &g, int vtype, int semiring, const int32_t *off,
                            const uint32_t *idx, const void *val, int32_t k, const void *X,
                            int64_t ldx, void *Y, int64_t ldy, const int32_t *wstart, int32_t win,
                            hipStream_t s) {
    if (k > g.kclass || win < 0 || (win > 0 && !wstart)) return hipErrorInvalidValue;
    switch (vtype) {
    case VAL_F64:
        return slab_by_semiring<double, double>(g, semiring, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case VAL_F32:
        return slab_by_semiring<float, float>(g, semiring, off, idx, val, k, X, ldx, Y, ldy, wstart, win, s);
    case VAL_BF16:
        return slab_by_semiring<uint16_t, float>(g, semiring, off, idx, val, k, X, ldx, Y, ldy, wstart,
                                                 win, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxe
