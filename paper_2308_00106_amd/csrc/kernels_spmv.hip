// CSR SpMV / SpMM kernels for gfx950 (Section 2: y_i = sum over row i of
// V[l] * x[COL[l]]), on (+, *) with FP64 accumulation for FP64 storage and
// FP32 accumulation for FP32 / BF16 storage.
//
// The product is bound by HBM bandwidth: each stored entry streams its value
// and column index once, x is gathered through L2, y is written once. The
// kernels therefore aim at coalesced val / col streams, enough memory-level
// parallelism, and keeping x resident in L2 (val, col and row_ptr are loaded
// non-temporally so the stream does not evict x).
//
// Variants (a variant id packs family and lanes per row):
//   GROUP  L lanes per row (L = 1 ... 64; rows per wavefront = 64 / L), rows
//          in storage order; lanes stride the row, then a butterfly reduction
//          over the L lanes.
//   BINNED rows grouped by length (bins of 1, 2, ... 64 lanes, built once per
//          matrix), one GROUP launch per non-empty bin over its row list.
//   MERGE  merge-path split of the row-end / nonzero sequence into equal
//          slices (Merrill and Garland, SC'16): every workgroup gets the same
//          work whatever the row lengths; row sums that cross a slice are
//          carried out and added by a fix-up pass in slice order.
//   FIXED  the rows split into 2048 equal contiguous parts, one workgroup
//          each, no counting (Section 7's equal-row parallel CSR).
//   COO    the coordinate form (Section 2): every stored entry carries its
//          row index; wavefronts take equal 256-entry tiles, reduce them by
//          row with a segmented scan, write whole rows directly and hand the
//          rows cut by a tile edge to a fix-up pass in tile order.
// Every variant sums each row in a fixed order, so results are deterministic.
#include "spmv_device.h"
#include "../../include/mxe.h"

#include <algorithm>

namespace mxe {

namespace {

constexpr int kBlock = 256;
constexpr int32_t kFixedParts = 256 * 8;     // FIXED: one part per resident workgroup slot

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Accumulate the entries of one row handled by this lane (lane, lane + L, ...),
// then reduce over the group of L lanes with xor butterflies: every lane ends
// with the same sum (addition is commutative), in a fixed order.
template <typename V, typename T, int L, int KM>
__device__ inline void row_dot(int32_t s, int32_t e, int lane, const int32_t *__restrict__ col,
                               const V *__restrict__ val, int32_t k, const T *__restrict__ X,
                               int64_t ldx, T (&acc)[KM]) {
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = T(0);
    int32_t p = s + lane;
    // two entries in flight per lane
    for (; p + L < e; p += 2 * L) {
        const int32_t c0 = ld_stream(col + p), c1 = ld_stream(col + p + L);
        const T a0 = ValLoad<V, T>::get(val + p), a1 = ValLoad<V, T>::get(val + p + L);
        const T *x0 = X + (int64_t)c0 * ldx, *x1 = X + (int64_t)c1 * ldx;
        if (KM == 1) {
            acc[0] += a0 * x0[0];
            acc[0] += a1 * x1[0];
        } else {
#pragma unroll
            for (int q = 0; q < KM; ++q)
                if (q < k) acc[q] += a0 * x0[q];
#pragma unroll
            for (int q = 0; q < KM; ++q)
                if (q < k) acc[q] += a1 * x1[q];
        }
    }
    if (p < e) {
        const int32_t c0 = ld_stream(col + p);
        const T a0 = ValLoad<V, T>::get(val + p);
        const T *x0 = X + (int64_t)c0 * ldx;
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (KM == 1 || q < k) acc[q] += a0 * x0[q];
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < KM; ++q) acc[q] += __shfl_xor(acc[q], off, L);
}

template <typename T, int L, int KM>
__device__ inline void store_row(T *__restrict__ Y, int64_t ldy, int32_t row, int lane, int32_t k,
                                 const T (&acc)[KM]) {
    T *y = Y + (int64_t)row * ldy;
    if (KM == 1) {
        if (lane == 0) y[0] = acc[0];
    } else {
        // spread the k stores over the group's lanes
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (q < k && (q % L) == lane) y[q] = acc[q];
    }
}

// Multi-RHS with column lanes (KM > 1, L >= KM): the row's L lanes are
// KM column lanes times L/KM entry lanes. The KM lanes of one entry read its
// value and column once (a broadcast) and the entry's X row as one contiguous
// KM-wide access, so a gather costs one request instead of KM; each lane keeps
// a single accumulator, reduced over the entry lanes of its column.
template <typename V, typename T, int L, int KM>
__device__ inline void row_product_cols(int32_t s, int32_t e, int lane,
                                        const int32_t *__restrict__ col,
                                        const V *__restrict__ val, int32_t k,
                                        const T *__restrict__ X, int64_t ldx,
                                        T *__restrict__ Y, int64_t ldy, int32_t row) {
    constexpr int E = L / KM;
    const int q = lane % KM, el = lane / KM;
    const bool active = q < k;
    T acc = T(0);
    int32_t p = s + el;
    for (; p + E < e; p += 2 * E) {            // two entries in flight per lane
        const int32_t c0 = ld_stream(col + p), c1 = ld_stream(col + p + E);
        const T a0 = ValLoad<V, T>::get(val + p), a1 = ValLoad<V, T>::get(val + p + E);
        const T x0 = active ? X[(int64_t)c0 * ldx + q] : T(0);
        const T x1 = active ? X[(int64_t)c1 * ldx + q] : T(0);
        acc += a0 * x0;
        acc += a1 * x1;
    }
    if (p < e) {
        const int32_t c0 = ld_stream(col + p);
        const T a0 = ValLoad<V, T>::get(val + p);
        acc += a0 * (active ? X[(int64_t)c0 * ldx + q] : T(0));
    }
#pragma unroll
    for (int off = L / 2; off >= KM; off >>= 1) acc += __shfl_xor(acc, off, L);
    if (el == 0 && active) Y[(int64_t)row * ldy + q] = acc;
}

// One row's product by its group of L lanes, written to Y.
template <typename V, typename T, int L, int KM>
__device__ inline void row_product(int32_t s, int32_t e, int lane, const int32_t *__restrict__ col,
                                   const V *__restrict__ val, int32_t k, const T *__restrict__ X,
                                   int64_t ldx, T *__restrict__ Y, int64_t ldy, int32_t row) {
    if constexpr (KM > 1 && L >= KM) {
        row_product_cols<V, T, L, KM>(s, e, lane, col, val, k, X, ldx, Y, ldy, row);
    } else {
        T acc[KM];
        row_dot<V, T, L, KM>(s, e, lane, col, val, k, X, ldx, acc);
        store_row<T, L, KM>(Y, ldy, row, lane, k, acc);
    }
}

// GROUP / BINNED: slot g (= global thread / L) computes row rows[g] (or g).
template <typename V, typename T, int L, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_group(
    int32_t count, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const V *__restrict__ val, int32_t k,
    const T *__restrict__ X, int64_t ldx, T *__restrict__ Y, int64_t ldy) {
    const int64_t slot = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
    const int lane = threadIdx.x % L;
    if (slot >= count) return;                  // whole groups leave together
    const int32_t row = rows ? rows[slot] : (int32_t)slot;
    const int32_t s = ld_stream(rp + row), e = ld_stream(rp + row + 1);
    row_product<V, T, L, KM>(s, e, lane, col, val, k, X, ldx, Y, ldy, row);
}

// ---- merge path -------------------------------------------------------------------

constexpr int kMergeIpt = 4;                          // path items per thread
constexpr int kMergeTile = kBlock * kMergeIpt;        // path items per workgroup

struct Coord { int32_t x, y; };                       // rows consumed, nonzeros consumed

// Largest x in [max(0, d - nnz), min(d, M)] whose row ends precede the
// nonzero at d - x: the merge of row_end[] = rp[1..M] with 0 .. nnz-1, where a
// row end sorts before a nonzero of equal index.
__device__ inline Coord merge_search(int64_t d, const int32_t *row_end, int32_t nrows,
                                     int64_t nnz) {
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < nrows ? d : nrows;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_end[mid] <= d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    return Coord{(int32_t)lo, (int32_t)(d - lo)};
}

__global__ __launch_bounds__(kBlock) void k_merge_coords(int32_t nrows, int64_t nnz,
                                                         const int32_t *__restrict__ rp,
                                                         int32_t ntiles, Coord *coords) {
    int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (w > ntiles) return;
    int64_t total = (int64_t)nrows + nnz;
    int64_t d = w * kMergeTile;
    if (d > total) d = total;
    coords[w] = merge_search(d, rp + 1, nrows, nnz);
}

struct Carry { int32_t row; int32_t pad; double v[4]; };   // row -1: none

// Each workgroup stages its slice's products and row ends in LDS with
// coalesced loads, walks the merge path in per-thread runs of kMergeIpt items,
// finishes rows spanning threads with a segmented scan in LDS, writes the rows
// that end inside the slice, and leaves the unfinished last row as a carry.
template <typename V, typename T, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_merge(
    int32_t nrows, int64_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, int32_t k, const T *__restrict__ X, int64_t ldx,
    T *__restrict__ Y, int64_t ldy, const Coord *__restrict__ coords, Carry *carry) {
    __shared__ T prod[kMergeTile][KM];
    __shared__ int32_t row_end[kMergeTile + 1];
    __shared__ int32_t key[kBlock];
    __shared__ T part[kBlock][KM];
    const Coord c0 = coords[blockIdx.x], c1 = coords[blockIdx.x + 1];
    const int32_t nrow_t = c1.x - c0.x, nnz_t = c1.y - c0.y;
    for (int i = threadIdx.x; i < nnz_t; i += kBlock) {
        const int32_t p = c0.y + i;
        const T a = ValLoad<V, T>::get(val + p);
        const T *xr = X + (int64_t)ld_stream(col + p) * ldx;
#pragma unroll
        for (int q = 0; q < KM; ++q) prod[i][q] = (KM == 1 || q < k) ? a * xr[q] : T(0);
    }
    for (int i = threadIdx.x; i < nrow_t; i += kBlock) row_end[i] = ld_stream(rp + c0.x + 1 + i);
    __syncthreads();
    // this thread's start on the slice's path
    const int32_t d = min((int32_t)threadIdx.x * kMergeIpt, nrow_t + nnz_t);
    int32_t lo = max(0, d - nnz_t), hi = min(d, nrow_t);
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (row_end[mid] - c0.y <= d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    int32_t tx = lo, ty = d - lo;
    T acc[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = T(0);
    int32_t first_done = -1;                          // first row this thread completes
    T first_val[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) first_val[q] = T(0);
    for (int it = 0; it < kMergeIpt; ++it) {
        if (tx < nrow_t && row_end[tx] - c0.y <= ty) {        // row end
            if (first_done < 0) {
                first_done = tx;
#pragma unroll
                for (int q = 0; q < KM; ++q) first_val[q] = acc[q];
            } else {
                T *y = Y + (int64_t)(c0.x + tx) * ldy;
#pragma unroll
                for (int q = 0; q < KM; ++q)
                    if (KM == 1 || q < k) y[q] = acc[q];
            }
#pragma unroll
            for (int q = 0; q < KM; ++q) acc[q] = T(0);
            ++tx;
        } else if (ty < nnz_t) {                               // nonzero
#pragma unroll
            for (int q = 0; q < KM; ++q) acc[q] += prod[ty][q];
            ++ty;
        }
    }
    // carry of this thread: the row it is inside at the end (tx), partial acc
    key[threadIdx.x] = tx;
#pragma unroll
    for (int q = 0; q < KM; ++q) part[threadIdx.x][q] = acc[q];
    __syncthreads();
    // inclusive segmented scan of the carries over threads with equal key
    for (int off = 1; off < kBlock; off <<= 1) {
        T v[KM];
        const bool take = (int)threadIdx.x >= off && key[threadIdx.x - off] == key[threadIdx.x];
#pragma unroll
        for (int q = 0; q < KM; ++q) v[q] = take ? part[threadIdx.x - off][q] : T(0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KM; ++q) part[threadIdx.x][q] += v[q];
        __syncthreads();
    }
    // the first row this thread completes began in earlier threads iff their
    // carry key equals it
    if (first_done >= 0) {
        if (threadIdx.x > 0 && key[threadIdx.x - 1] == first_done) {
#pragma unroll
            for (int q = 0; q < KM; ++q) first_val[q] = part[threadIdx.x - 1][q] + first_val[q];
        }
        T *y = Y + (int64_t)(c0.x + first_done) * ldy;
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (KM == 1 || q < k) y[q] = first_val[q];
    }
    // slice carry: the last thread's scanned partial for the row still open at
    // the slice end. Once every row end of the slice is consumed that row is
    // local index nrow_t, i.e. the next slice's first row c1.x.
    if (threadIdx.x == kBlock - 1) {
        Carry cr;
        const int32_t open_row = c0.x + key[kBlock - 1];
        cr.row = open_row < nrows ? open_row : -1;
        cr.pad = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) cr.v[q] = q < KM ? (double)part[kBlock - 1][q] : 0.0;
        carry[blockIdx.x] = cr;
    }
}

// Rows crossing slices: the slice where the row ends wrote its own part;
// add the carries of the earlier slices, in slice order.
template <typename T, int KM>
__global__ __launch_bounds__(kBlock) void k_merge_fixup(int32_t ntiles, const Carry *carry,
                                                        int32_t k, T *__restrict__ Y,
                                                        int64_t ldy) {
    int32_t w = blockIdx.x * kBlock + threadIdx.x;
    if (w >= ntiles) return;
    const int32_t row = carry[w].row;
    if (row < 0) return;
    if (w > 0 && carry[w - 1].row == row) return;        // not the first carry of this row
    // carries are partial sums in T; add them in T in slice order
    T t[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) t[q] = T(0);
    for (int32_t u = w; u < ntiles && carry[u].row == row; ++u)
#pragma unroll
        for (int q = 0; q < KM; ++q) t[q] += (T)carry[u].v[q];
    T *y = Y + (int64_t)row * ldy;
#pragma unroll
    for (int q = 0; q < KM; ++q)
        if (KM == 1 || q < k) y[q] = t[q] + y[q];
}

// FIXED: the equal-row split of Section 7's parallel CSR on the GPU. A fixed
// grid of P workgroups; workgroup w owns rows [w M / P, (w + 1) M / P) and
// nothing rebalances them, so a cluster of heavy rows makes laggards unless
// a random row permutation has spread it (the paper's load-balance argument,
// Section 1).
template <typename V, typename T>
__global__ __launch_bounds__(kBlock) void k_spmv_fixed(int32_t nrows, int32_t parts,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const V *__restrict__ val, int32_t k,
                                                       const T *__restrict__ X, int64_t ldx,
                                                       T *__restrict__ Y, int64_t ldy, int L,
                                                       int KM) {
    const int64_t w = blockIdx.x;
    const int32_t r0 = (int32_t)(w * nrows / parts), r1 = (int32_t)((w + 1) * nrows / parts);
    rows_runtime<V, T, kBlock>(rp, col, val, k, X, ldx, Y, ldy, L, KM, r0, r1, threadIdx.x);
}

// ---- COO -------------------------------------------------------------------------

constexpr int kCooTile = 256;                 // entries per wavefront tile

__global__ __launch_bounds__(kBlock) void k_coo_rows(int32_t nrows, const int32_t *__restrict__ rp,
                                                     int32_t *__restrict__ row) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) row[e] = (int32_t)i;
}

template <typename T, int KM>
__global__ __launch_bounds__(kBlock) void k_zero_rows(int32_t nrows, int32_t k, T *__restrict__ Y,
                                                      int64_t ldy) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)nrows * k;
         i += (int64_t)gridDim.x * blockDim.x)
        Y[(i / k) * ldy + i % k] = T(0);
}

// Tile t = entries [e0, e1). Its first row is a "head" carried out when it
// began in an earlier tile; its last row is a "tail" carried out when it goes
// on into the next tile (and is not that head). Every other row lies wholly
// in the tile and is written here, together with the empty rows that follow
// it. crow[2t], crow[2t+1] = head / tail row or -1; cval holds their partial
// sums (KM values each).
template <typename V, typename T, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_coo(int32_t nrows, int64_t nnz,
                                                     const int32_t *__restrict__ row,
                                                     const int32_t *__restrict__ col,
                                                     const V *__restrict__ val, int32_t k,
                                                     const T *__restrict__ X, int64_t ldx,
                                                     T *__restrict__ Y, int64_t ldy,
                                                     int32_t *__restrict__ crow,
                                                     T *__restrict__ cval) {
    const int lane = threadIdx.x % kWave;
    const int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t e0 = t * kCooTile;
    if (e0 >= nnz) return;                                     // uniform per wavefront
    const int64_t e1 = e0 + kCooTile < nnz ? e0 + kCooTile : nnz;
    const int32_t head_row = row[e0], last_row = row[e1 - 1];
    const bool head_valid = e0 > 0 && row[e0 - 1] == head_row;
    const bool tail_valid = e1 < nnz && row[e1] == last_row && !(head_valid && head_row == last_row);
    if (lane == 0) {
        crow[2 * t] = head_valid ? head_row : -1;
        crow[2 * t + 1] = tail_valid ? last_row : -1;
    }
    if (t == 0)                                                // empty rows before the first entry
        for (int32_t r = lane; r < head_row; r += kWave)
            for (int q = 0; q < KM; ++q)
                if (KM == 1 || q < k) Y[(int64_t)r * ldy + q] = T(0);
    int32_t carry_row = -1;                                    // row running on from the last chunk
    T carry[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) carry[q] = T(0);
    for (int64_t base = e0; base < e1; base += kWave) {       // uniform per wavefront
        const int64_t e = base + lane;
        const bool valid = e < e1;
        uint32_t key = 0xffffffffu;
        int32_t nr = 0;
        T prod[KM];
        if (valid) {
            key = (uint32_t)ld_stream(row + e);
            nr = e + 1 < nnz ? row[e + 1] : nrows;
            const T a = ValLoad<V, T>::get(val + e);
            const T *xr = X + (int64_t)ld_stream(col + e) * ldx;
#pragma unroll
            for (int q = 0; q < KM; ++q) prod[q] = (KM == 1 || q < k) ? a * xr[q] : T(0);
        } else {
#pragma unroll
            for (int q = 0; q < KM; ++q) prod[q] = T(0);
        }
        if (lane == 0 && carry_row >= 0 && (uint32_t)carry_row == key) {
#pragma unroll
            for (int q = 0; q < KM; ++q) prod[q] += carry[q];
        }
        segmented_scan<T, KM>(key, prod);                      // inclusive, by row
        const uint32_t nxt = __shfl_down(key, 1);
        const bool seg_end = valid && (lane == kWave - 1 || nxt != key);
        const bool to_next = seg_end && e + 1 < e1 && nr == (int32_t)key;
        carry_row = __shfl(to_next ? (int32_t)key : -1, kWave - 1);
#pragma unroll
        for (int q = 0; q < KM; ++q) carry[q] = __shfl(prod[q], kWave - 1);
        if (seg_end && !to_next) {
            const int32_t r = (int32_t)key;
            if (head_valid && r == head_row) {
#pragma unroll
                for (int q = 0; q < KM; ++q) cval[(2 * t) * KM + q] = prod[q];
            } else if (tail_valid && e == e1 - 1) {
#pragma unroll
                for (int q = 0; q < KM; ++q) cval[(2 * t + 1) * KM + q] = prod[q];
            } else {
#pragma unroll
                for (int q = 0; q < KM; ++q)
                    if (KM == 1 || q < k) Y[(int64_t)r * ldy + q] = prod[q];
            }
            for (int32_t z = r + 1; z < nr; ++z)               // empty rows up to the next entry's
#pragma unroll
                for (int q = 0; q < KM; ++q)
                    if (KM == 1 || q < k) Y[(int64_t)z * ldy + q] = T(0);
        }
    }
}

// Each row cut by tile edges is owned by the tile where it starts (its tail):
// that tile's partial, then the heads of the following tiles in order.
template <typename T, int KM>
__global__ __launch_bounds__(kBlock) void k_coo_fixup(int64_t ntiles, const int32_t *__restrict__ crow,
                                                      const T *__restrict__ cval, int32_t k,
                                                      T *__restrict__ Y, int64_t ldy) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = crow[2 * t + 1];
        if (r < 0) continue;
        T sum[KM];
#pragma unroll
        for (int q = 0; q < KM; ++q) sum[q] = cval[(2 * t + 1) * KM + q];
        for (int64_t u = t + 1; u < ntiles && crow[2 * u] == r; ++u)
#pragma unroll
            for (int q = 0; q < KM; ++q) sum[q] += cval[(2 * u) * KM + q];
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (KM == 1 || q < k) Y[(int64_t)r * ldy + q] = sum[q];
    }
}

template <typename V, typename T, int KM>
hipError_t coo_launch(const SpmvArgs &a, hipStream_t s) {
    if (!a.coo_row || !a.carry_ws) return hipErrorInvalidValue;
    if (a.nnz == 0) {
        hipLaunchKernelGGL((k_zero_rows<T, KM>), dim3((unsigned)std::min<int64_t>(cdiv((int64_t)a.nrows * a.k, kBlock), 4096)),
                           dim3(kBlock), 0, s, a.nrows, a.k, (T *)a.Y, a.ldy);
        return hipGetLastError();
    }
    const int64_t ntiles = cdiv(a.nnz, kCooTile);
    int32_t *crow = (int32_t *)a.carry_ws;
    T *cval = (T *)((char *)a.carry_ws + ((sizeof(int32_t) * 2 * ntiles + 255) & ~size_t(255)));
    hipLaunchKernelGGL((k_spmv_coo<V, T, KM>), dim3((unsigned)cdiv(ntiles, kBlock / kWave)),
                       dim3(kBlock), 0, s, a.nrows, a.nnz, a.coo_row, a.col, (const V *)a.val, a.k,
                       (const T *)a.X, a.ldx, (T *)a.Y, a.ldy, crow, cval);
    hipLaunchKernelGGL((k_coo_fixup<T, KM>), dim3((unsigned)std::min<int64_t>(cdiv(ntiles, kBlock), 4096)),
                       dim3(kBlock), 0, s, ntiles, (const int32_t *)crow, (const T *)cval, a.k,
                       (T *)a.Y, a.ldy);
    return hipGetLastError();
}

// ---- other semirings (Section 2) --------------------------------------------------
// L lanes per row take its entries in a lane stride and combine them with the
// semiring's product, then an xor butterfly over the L lanes with its sum
// (Semiring in device_common.h). min and or are exact, so the order of the
// terms does not matter.

template <typename V, typename T, int SR, int L, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_semiring(int32_t nrows, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col,
                                                          const V *__restrict__ val, int32_t k,
                                                          const T *__restrict__ X, int64_t ldx,
                                                          T *__restrict__ Y, int64_t ldy) {
    using S = Semiring<SR, T>;
    const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const int64_t row = gt / L;
    const int lane = (int)(gt % L);
    T acc[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) acc[q] = S::identity();
    if (row < nrows) {                       // other lanes still join the butterfly
        for (int32_t p = rp[row] + lane; p < rp[row + 1]; p += L) {
            const T a = ValLoad<V, T>::get(val + p);
            const T *xr = X + (int64_t)ld_stream(col + p) * ldx;
#pragma unroll
            for (int q = 0; q < KM; ++q)
                if (KM == 1 || q < k) acc[q] = S::add(acc[q], S::mul(a, xr[q]));
        }
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < KM; ++q) acc[q] = S::add(acc[q], __shfl_xor(acc[q], off));
    if (row < nrows && lane == 0)
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (KM == 1 || q < k) Y[row * ldy + q] = acc[q];
}

template <typename V, typename T, int SR, int L>
hipError_t semiring_by_k(const SpmvArgs &a, hipStream_t s) {
    const int64_t grid = cdiv((int64_t)a.nrows * L, kBlock);
#define MXE_SR_LAUNCH(KMV)                                                                         \
    hipLaunchKernelGGL((k_spmv_semiring<V, T, SR, L, KMV>), dim3((unsigned)grid), dim3(kBlock), 0, \
                       s, a.nrows, a.rp, a.col, (const V *)a.val, a.k, (const T *)a.X, a.ldx,      \
                       (T *)a.Y, a.ldy)
    if (a.k <= 1) MXE_SR_LAUNCH(1);
    else if (a.k <= 4) MXE_SR_LAUNCH(4);
    else MXE_SR_LAUNCH(16);
#undef MXE_SR_LAUNCH
    return hipGetLastError();
}

template <typename V, typename T, int SR>
hipError_t semiring_by_lanes(const SpmvArgs &a, hipStream_t s) {
    const bool long_rows = a.nrows > 0 && a.nnz / a.nrows > 16;
    return long_rows ? semiring_by_k<V, T, SR, 32>(a, s) : semiring_by_k<V, T, SR, 8>(a, s);
}

template <int SR>
hipError_t semiring_by_type(const SpmvArgs &a, hipStream_t s) {
    switch (a.vtype) {
    case VAL_F64: return semiring_by_lanes<double, double, SR>(a, s);
    case VAL_F32: return semiring_by_lanes<float, float, SR>(a, s);
    case VAL_BF16: return semiring_by_lanes<uint16_t, float, SR>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// ---- launch helpers ---------------------------------------------------------------------

template <typename V, typename T, int L, int KM>
void group_launch(const SpmvArgs &a, const int32_t *rows, int32_t count, hipStream_t s) {
    const int64_t threads = (int64_t)count * L;
    const int grid = (int)cdiv(threads, kBlock);
    hipLaunchKernelGGL((k_spmv_group<V, T, L, KM>), dim3(grid), dim3(kBlock), 0, s, count, rows,
                       a.rp, a.col, (const V *)a.val, a.k, (const T *)a.X, a.ldx, (T *)a.Y, a.ldy);
}

template <typename V, typename T, int KM>
hipError_t group_by_lanes(const SpmvArgs &a, int lanes, const int32_t *rows, int32_t count,
                          hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (lanes) {
    case 1: group_launch<V, T, 1, KM>(a, rows, count, s); break;
    case 2: group_launch<V, T, 2, KM>(a, rows, count, s); break;
    case 4: group_launch<V, T, 4, KM>(a, rows, count, s); break;
    case 8: group_launch<V, T, 8, KM>(a, rows, count, s); break;
    case 16: group_launch<V, T, 16, KM>(a, rows, count, s); break;
    case 32: group_launch<V, T, 32, KM>(a, rows, count, s); break;
    case 64: group_launch<V, T, 64, KM>(a, rows, count, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline int32_t merge_tiles(int32_t nrows, int64_t nnz) {
    return (int32_t)std::max<int64_t>(1, cdiv((int64_t)nrows + nnz, kMergeTile));
}

// coords: the matrix's slice starts (launch_merge_coords, read only here);
// the carries live in the launch's own workspace, so launches of one matrix
// on different streams never share them
template <typename V, typename T, int KM>
hipError_t merge_launch(const SpmvArgs &a, hipStream_t s) {
    if (!a.merge_coords || !a.carry_ws) return hipErrorInvalidValue;
    const int32_t ntiles = merge_tiles(a.nrows, a.nnz);
    const Coord *coords = (const Coord *)a.merge_coords;
    Carry *carry = (Carry *)a.carry_ws;
    hipLaunchKernelGGL((k_spmv_merge<V, T, KM>), dim3(ntiles), dim3(kBlock), 0, s, a.nrows, a.nnz,
                       a.rp, a.col, (const V *)a.val, a.k, (const T *)a.X, a.ldx, (T *)a.Y, a.ldy,
                       (const Coord *)coords, carry);
    hipLaunchKernelGGL((k_merge_fixup<T, KM>), dim3(cdiv(ntiles, kBlock)), dim3(kBlock), 0, s,
                       ntiles, (const Carry *)carry, a.k, (T *)a.Y, a.ldy);
    return hipGetLastError();
}

template <typename V, typename T, int KM>
hipError_t spmv_k(const SpmvArgs &a, int variant, hipStream_t s) {
    const int family = variant & 0xf00, lanes = variant & 0xff;
    if (family == MXE_VAR_GROUP) return group_by_lanes<V, T, KM>(a, lanes, nullptr, a.nrows, s);
    if (family == MXE_VAR_BINNED) {
        for (int b = 0; b < kNumBins; ++b) {
            const int32_t n = a.bin_off_host[b + 1] - a.bin_off_host[b];
            hipError_t e = group_by_lanes<V, T, KM>(a, 1 << b, a.bin_list + a.bin_off_host[b], n, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (family == MXE_VAR_MERGE) {
        if constexpr (KM <= 4) return merge_launch<V, T, KM>(a, s);
        return hipErrorInvalidValue;
    }
    if (family == MXE_VAR_COO) return coo_launch<V, T, KM>(a, s);
    if (family == MXE_VAR_FIXED) {
        const int L = std::max(lanes, KM);
        const int32_t parts = kFixedParts;
        hipLaunchKernelGGL((k_spmv_fixed<V, T>), dim3(parts), dim3(kBlock), 0, s, a.nrows, parts,
                           a.rp, a.col, (const V *)a.val, a.k, (const T *)a.X, a.ldx, (T *)a.Y,
                           a.ldy, L, KM);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <typename V, typename T>
hipError_t spmv_t(const SpmvArgs &a, int variant, hipStream_t s) {
    if (a.k <= 1) return spmv_k<V, T, 1>(a, variant, s);
    if (a.k <= 2) return spmv_k<V, T, 2>(a, variant, s);
    if (a.k <= 4) return spmv_k<V, T, 4>(a, variant, s);
    if (a.k <= 8) return spmv_k<V, T, 8>(a, variant, s);
    if (a.k <= 16) return spmv_k<V, T, 16>(a, variant, s);
    return hipErrorInvalidValue;
}

}  // namespace

size_t merge_coords_bytes(int32_t nrows, int64_t nnz) {
    return sizeof(Coord) * ((size_t)merge_tiles(nrows, nnz) + 1);
}

size_t merge_carry_bytes(int32_t nrows, int64_t nnz) {
    return sizeof(Carry) * (size_t)merge_tiles(nrows, nnz);
}

hipError_t launch_merge_coords(int32_t nrows, int64_t nnz, const int32_t *rp, void *coords,
                               hipStream_t s) {
    const int32_t ntiles = merge_tiles(nrows, nnz);
    hipLaunchKernelGGL(k_merge_coords, dim3(cdiv(ntiles + 1, kBlock)), dim3(kBlock), 0, s, nrows,
                       nnz, rp, ntiles, (Coord *)coords);
    return hipGetLastError();
}

hipError_t launch_spmv_semiring(const SpmvArgs &a, int semiring, hipStream_t s) {
    if (a.nrows <= 0) return hipSuccess;
    if (a.k < 1 || a.k > 16) return hipErrorInvalidValue;
    switch (semiring) {
    case MXE_SR_MIN_PLUS: return semiring_by_type<MXE_SR_MIN_PLUS>(a, s);
    case MXE_SR_OR_AND: return semiring_by_type<MXE_SR_OR_AND>(a, s);
    default: return hipErrorInvalidValue;
    }
}

size_t coo_ws_bytes(int64_t nnz, int kclass, int elem_bytes) {
    const int64_t ntiles = std::max<int64_t>(1, cdiv(nnz, kCooTile));
    return ((sizeof(int32_t) * 2 * ntiles + 255) & ~size_t(255)) +
           (size_t)elem_bytes * 2 * ntiles * kclass;
}

hipError_t launch_coo_rows(int32_t nrows, const int32_t *rp, int32_t *row, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coo_rows, dim3((unsigned)std::min<int64_t>(cdiv(nrows, kBlock), 16384)),
                       dim3(kBlock), 0, s, nrows, rp, row);
    return hipGetLastError();
}

hipError_t launch_spmv(const SpmvArgs &a, int variant, hipStream_t s) {
    if (a.nrows <= 0) return hipSuccess;
    if ((variant & 0xf00) == MXE_VAR_SLAB || (variant & 0xf00) == MXE_VAR_WINDOW) {
        if (!a.slab) return hipErrorInvalidValue;
        const bool win = (variant & 0xf00) == MXE_VAR_WINDOW;
        if (win && (!a.slab_wstart || a.slab_win < 1)) return hipErrorInvalidValue;
        return launch_spmv_slab(*a.slab, a.vtype, MXE_SR_PLUS_TIMES, a.slab_off, a.slab_idx,
                                a.slab_val, a.k, a.X, a.ldx, a.Y, a.ldy, win ? a.slab_wstart : nullptr,
                                win ? a.slab_win : 0, s);
    }
    switch (a.vtype) {
    case VAL_F64: return spmv_t<double, double>(a, variant, s);
    case VAL_F32: return spmv_t<float, float>(a, variant, s);
    case VAL_BF16: return spmv_t<uint16_t, float>(a, variant, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxe
