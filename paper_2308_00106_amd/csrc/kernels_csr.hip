// Random permutation, permuted CSR construction, vector permutes, scans,
// row-length bins and value conversion for gfx950 (wave64).
//
// The random permutation (Section 3; Eq. 1) is the stable ascending order of
// 64-bit SplitMix64 keys. Because the keys are a pure function of the index,
// they are never stored. Up to 8.4M indices, an LDS radix pass buckets the
// indices by the top 10-12 key bits (per-workgroup LDS histograms, a scan,
// an LDS-cursor scatter of 4-byte indices) and one workgroup per bucket of
// ~2K sorts it in LDS (split by the next 8 bits, then a rank by (key, index)
// inside sub-buckets of ~8). Larger ranges bucket by up to 20 top bits with
// device atomics instead of LDS histograms and sort the buckets the same way.
// Either way two light passes over 4-byte indices replace the eight read-write
// passes of an LSD radix sort over 12-byte (key, index) pairs.
#include "device_common.h"
#include "internal.h"

namespace mxe {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;                          // per thread
constexpr int kScanTile = kBlock * kScanItems;         // 2048 per workgroup

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline int grid_for(int64_t n, int per_block = kBlock, int64_t cap = 1 << 20) {
    int64_t g = cdiv(n, per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ---- fills -------------------------------------------------------------------

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_i32(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// ---- block-level exclusive scan of one int per thread ----------------------

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *wsum, int32_t *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int32_t inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) woff += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    if (total) *total = tot;
    return inc - v + woff;
}

// ---- three-phase exclusive scan ---------------------------------------------

__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(const int32_t *in, int64_t n,
                                                           int32_t *sums) {
    __shared__ int32_t wsum[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t acc = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        int64_t i = base + t * kBlock + threadIdx.x;
        if (i < n) acc += in[i];
    }
    int32_t tot;
    block_exclusive_scan(acc, wsum, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup scans the tile sums in place (exclusive).
__global__ __launch_bounds__(kBlock) void k_scan_sums(int32_t *sums, int64_t ntiles) {
    __shared__ int32_t wsum[kBlock / kWave];
    int32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kBlock) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < ntiles ? sums[i] : 0;
        int32_t tot;
        int32_t ex = block_exclusive_scan(v, wsum, &tot);
        if (i < ntiles) sums[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t *in, int32_t *out,
                                                       int64_t n, const int32_t *sums) {
    __shared__ int32_t tile[kScanTile];
    __shared__ int32_t wsum[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        int64_t i = base + t * kBlock + threadIdx.x;
        tile[t * kBlock + threadIdx.x] = i < n ? in[i] : 0;
    }
    __syncthreads();
    int32_t loc[kScanItems];
    int32_t acc = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        loc[t] = acc;
        acc += tile[threadIdx.x * kScanItems + t];
    }
    int32_t ex = block_exclusive_scan(acc, wsum, nullptr) + sums[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) tile[threadIdx.x * kScanItems + t] = loc[t] + ex;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        int64_t i = base + t * kBlock + threadIdx.x;
        if (i < n) out[i] = tile[t * kBlock + threadIdx.x];
    }
}

// ---- random permutation: global bucketing (above 8.4M indices) ---------------

inline int bucket_bits(int64_t n) {          // mean bucket <= 2048 up to 2^31 indices
    int b = 0;
    while (b < 20 && (n >> b) > 2048) ++b;
    return b;
}

__device__ inline uint32_t bucket_of(uint64_t key, int bits) {
    return bits == 0 ? 0u : (uint32_t)(key >> (64 - bits));
}

__global__ __launch_bounds__(kBlock) void k_bucket_count(int64_t n, uint64_t seed, int bits,
                                                         int32_t *counts, int32_t *slot) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = bucket_of(sm64_key(seed, (uint64_t)i), bits);
        slot[i] = atomicAdd(&counts[b], 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_bucket_scatter(int64_t n, uint64_t seed, int bits,
                                                           const int32_t *offsets,
                                                           const int32_t *slot, int32_t *items) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = bucket_of(sm64_key(seed, (uint64_t)i), bits);
        items[offsets[b] + slot[i]] = (int32_t)i;
    }
}

// LDS radix path (n up to kLdsPermMax): keys are bucketed by their top
// `bits` bits with per-workgroup LDS histograms (no device-wide atomics), then
// one workgroup per bucket splits it by the next kSubBits bits in LDS and
// ranks every item by (key, index) inside its sub-bucket, a handful of items.
constexpr int kPermItems = 8192;                         // indices per bucketing workgroup
constexpr int kPermMaxBits = 12;                         // at most 4096 buckets
constexpr int kPermMeanBucket = 2048;
constexpr int kBucketCap = 4096;                         // items a workgroup sorts in LDS
constexpr int kSubBits = 8;                              // sub-buckets = kBlock
constexpr int64_t kLdsPermMax = (int64_t)kPermMeanBucket << kPermMaxBits;

inline int radix_bits(int64_t n) {                       // mean bucket <= kPermMeanBucket
    int b = 0;
    while (b < kPermMaxBits && (n >> b) > kPermMeanBucket) ++b;
    return b;
}

__device__ inline uint32_t top_digit(uint64_t key, int bits) {
    return bits == 0 ? 0u : (uint32_t)(key >> (64 - bits));
}
__device__ inline uint32_t sub_digit(uint64_t key, int bits) {
    return (uint32_t)(key >> (64 - bits - kSubBits)) & ((1u << kSubBits) - 1u);
}

// counts[d * nwg + w] = items of workgroup w's index range in bucket d
__global__ __launch_bounds__(kBlock) void k_perm_count(int64_t n, uint64_t seed, int bits,
                                                       int32_t nwg, int32_t *counts) {
    extern __shared__ int32_t hist[];
    const int nd = 1 << bits;
    for (int d = threadIdx.x; d < nd; d += kBlock) hist[d] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPermItems;
    const int64_t i1 = i0 + kPermItems < n ? i0 + kPermItems : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock)
        atomicAdd(&hist[top_digit(sm64_key(seed, (uint64_t)i), bits)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += kBlock) counts[(int64_t)d * nwg + blockIdx.x] = hist[d];
}

// offsets: the exclusive scan of counts; items[pos] = index, in any order
// inside a bucket (the bucket sort fixes the order)
__global__ __launch_bounds__(kBlock) void k_perm_scatter(int64_t n, uint64_t seed, int bits,
                                                         int32_t nwg, const int32_t *offsets,
                                                         int32_t *items) {
    extern __shared__ int32_t cursor[];
    const int nd = 1 << bits;
    for (int d = threadIdx.x; d < nd; d += kBlock) cursor[d] = offsets[(int64_t)d * nwg + blockIdx.x];
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPermItems;
    const int64_t i1 = i0 + kPermItems < n ? i0 + kPermItems : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int32_t pos = atomicAdd(&cursor[top_digit(sm64_key(seed, (uint64_t)i), bits)], 1);
        items[pos] = (int32_t)i;
    }
}

__device__ inline bool key_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// One workgroup per bucket: final position of each item = bucket start +
// start of its sub-bucket + its rank by (key, index) inside the sub-bucket.
// A bucket above kBucketCap (not expected from uniform keys) is ranked
// against the whole bucket in memory instead.
// Bucket d spans items [offsets[d * stride], offsets[(d + 1) * stride]).
__global__ __launch_bounds__(kBlock) void k_perm_bucket_sort(int32_t nd, int32_t stride, uint64_t seed,
                                                             int bits, const int32_t *offsets,
                                                             const int32_t *items, int32_t *perm,
                                                             int32_t *inv) {
    __shared__ uint64_t skey[kBucketCap];
    __shared__ int32_t sidx[kBucketCap];
    __shared__ int32_t sub[kBlock + 1];
    __shared__ int32_t cursor[kBlock];
    __shared__ int32_t wsum[kBlock / kWave];
    const int32_t d = blockIdx.x;
    const int32_t o = offsets[(int64_t)d * stride];
    const int32_t m = offsets[(int64_t)(d + 1) * stride] - o;   // the scan's last entry is n
    if (m > kBucketCap) {
        for (int32_t t = threadIdx.x; t < m; t += kBlock) {
            const int32_t idx = items[o + t];
            const uint64_t key = sm64_key(seed, (uint64_t)idx);
            int32_t r = 0;
            for (int32_t u = 0; u < m; ++u) {
                const int32_t iu = items[o + u];
                r += key_less(sm64_key(seed, (uint64_t)iu), iu, key, idx);
            }
            perm[o + r] = idx;
            if (inv) inv[idx] = o + r;
        }
        return;
    }
    sub[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < m; t += kBlock)
        atomicAdd(&sub[sub_digit(sm64_key(seed, (uint64_t)items[o + t]), bits)], 1);
    __syncthreads();
    int32_t total;
    const int32_t ex = block_exclusive_scan(sub[threadIdx.x], wsum, &total);
    sub[threadIdx.x] = ex;
    cursor[threadIdx.x] = ex;
    if (threadIdx.x == 0) sub[kBlock] = total;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < m; t += kBlock) {
        const int32_t idx = items[o + t];
        const uint64_t key = sm64_key(seed, (uint64_t)idx);
        const int32_t p = atomicAdd(&cursor[sub_digit(key, bits)], 1);
        skey[p] = key;
        sidx[p] = idx;
    }
    __syncthreads();
    for (int32_t p = threadIdx.x; p < m; p += kBlock) {
        const uint64_t key = skey[p];
        const int32_t idx = sidx[p];
        const uint32_t sd = sub_digit(key, bits);
        const int32_t b0 = sub[sd], b1 = sub[sd + 1];
        int32_t r = 0;
        for (int32_t q = b0; q < b1; ++q) r += key_less(skey[q], sidx[q], key, idx);
        perm[o + b0 + r] = idx;
        if (inv) inv[idx] = o + b0 + r;
    }
}

// ---- permuted CSR --------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_perm_row_len(int32_t nrows, const int32_t *rp,
                                                         const int32_t *rperm, int32_t *len) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nrows) {
        int32_t src = rperm[i];
        len[i] = rp[src + 1] - rp[src];
    } else if (i == nrows) {
        len[i] = 0;
    }
}

constexpr int kSortRows = 16;                           // rows of A per wavefront
constexpr int kSortStage = 1024;                        // staged entries per wavefront
constexpr int kSortWaves = kBlock / kWave;

// Each wavefront moves kSortRows consecutive rows of A (row i goes to row
// rinv[i] of B, at rp_b[rinv[i]]): it stages the rows' relabelled columns
// (j -> cinv[j]) in LDS, then every lane takes entries, finds each one's row
// by binary search over the staged row starts, and writes it at its rank among
// its row's new columns (distinct, so the rank is its sorted position). Reads
// stream through A in order, so a matrix whose columns cluster by row keeps
// its cinv lookups in cache. Groups of rows with more than kSortStage entries
// are moved one row at a time; a row longer than the stage ranks against
// cinv in memory.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_gather_relabel_sort(
    int32_t nrows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const int32_t *__restrict__ rinv, const int32_t *__restrict__ cinv,
    const int32_t *__restrict__ rp_b, int32_t *__restrict__ col_b, V *__restrict__ val_b) {
    __shared__ int32_t stage[kSortWaves][kSortStage];
    __shared__ int32_t rstart[kSortWaves][kSortRows + 1];   // row starts, relative to e0
    __shared__ int32_t rdest[kSortWaves][kSortRows];        // where each row goes in B
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t r0 = ((int64_t)blockIdx.x * kSortWaves + wave) * kSortRows;
    if (r0 >= nrows) return;                            // uniform per wavefront
    const int nr = (int)std::min<int64_t>(kSortRows, nrows - r0);
    const int32_t e0 = rp[r0];
    if (lane <= nr) rstart[wave][lane] = rp[r0 + lane] - e0;
    if (lane < nr) rdest[wave][lane] = rp_b[rinv[r0 + lane]];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int32_t n = rstart[wave][nr];
    auto relabel = [&](int32_t j) { return cinv ? cinv[j] : j; };
    if (n <= kSortStage) {
        for (int32_t i = lane; i < n; i += kWave) stage[wave][i] = relabel(col[e0 + i]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int32_t i = lane; i < n; i += kWave) {
            int lo = 0, hi = nr - 1;                    // last row whose start is <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rstart[wave][mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            const int32_t b = rstart[wave][lo], e = rstart[wave][lo + 1];
            const int32_t c = stage[wave][i];
            int32_t r = i - b;                          // rows only: order unchanged
            if (cinv) {
                r = 0;
                for (int32_t u = b; u < e; ++u) r += stage[wave][u] < c;
            }
            col_b[rdest[wave][lo] + r] = c;
            val_b[rdest[wave][lo] + r] = val[e0 + i];
        }
        return;
    }
    for (int j = 0; j < nr; ++j) {                      // one row at a time
        const int32_t b = e0 + rstart[wave][j], len = rstart[wave][j + 1] - rstart[wave][j];
        const int32_t d0 = rdest[wave][j];
        const bool staged = len <= kSortStage;
        if (staged)
            for (int32_t t = lane; t < len; t += kWave) stage[wave][t] = relabel(col[b + t]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int32_t t = lane; t < len; t += kWave) {
            const int32_t c = staged ? stage[wave][t] : relabel(col[b + t]);
            int32_t r = t;
            if (cinv) {
                r = 0;
                if (staged) {
                    for (int32_t u = 0; u < len; ++u) r += stage[wave][u] < c;
                } else {
                    for (int32_t u = 0; u < len; ++u) r += cinv[col[b + u]] < c;
                }
            }
            col_b[d0 + r] = c;
            val_b[d0 + r] = val[b + t];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---- vector permutes (Eq. 1) -----------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_rows(int32_t n, int32_t k,
                                                        const int32_t *__restrict__ perm,
                                                        const T *__restrict__ X, int64_t ldx,
                                                        T *__restrict__ Xp, int64_t ldxp) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const T *src = X + (int64_t)perm[j] * ldx;
        T *dst = Xp + j * ldxp;
        for (int32_t c = 0; c < k; ++c) dst[c] = src[c];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_rows(int32_t n, int32_t k,
                                                         const int32_t *__restrict__ perm,
                                                         const T *__restrict__ Yp, int64_t ldyp,
                                                         T *__restrict__ Y, int64_t ldy) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T *src = Yp + i * ldyp;
        T *dst = Y + (int64_t)perm[i] * ldy;
        for (int32_t c = 0; c < k; ++c) dst[c] = src[c];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_cols(int32_t n, int32_t k, const T *__restrict__ src,
                                                      int64_t lds, T *__restrict__ dst,
                                                      int64_t ldd) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t c = 0; c < k; ++c) dst[i * ldd + c] = src[i * lds + c];
}

// Several column blocks at once: entry blockIdx.y of the table copies its
// source's k columns into columns [c0, c0 + k) of its destination, rows
// [0, n); the grid's x dimension strides over the n x k elements, one per
// thread in row-major order, so neighbouring threads touch neighbouring
// addresses on both sides.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_cols(const PackCols *__restrict__ table) {
    const PackCols e = table[blockIdx.y];
    const T *src = as_global((const T *)e.src);
    T *dst = as_global((T *)e.dst) + e.c0;
    const int64_t total = (int64_t)e.n * e.k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / e.k;
        const int32_t c = (int32_t)(i - r * e.k);
        dst[r * e.ldd + c] = src[r * e.lds + c];
    }
}

// ---- value conversion --------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_f64_to_f32(const double *in, float *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];                 // v_cvt_f32_f64: round to nearest even
}

__global__ __launch_bounds__(kBlock) void k_f64_to_bf16(const double *in, uint16_t *out,
                                                        int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = bf16_from_f64(in[i]);
}

// ---- row statistics and bins ------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_row_max(int32_t nrows, const int32_t *rp,
                                                    int32_t *max_len) {
    int32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, rp[i + 1] - rp[i]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(max_len, m);
}

__global__ __launch_bounds__(kBlock) void k_bin_count(int32_t nrows, const int32_t *rp,
                                                      int32_t *cnt, int32_t nwg) {
    __shared__ int32_t c[kNumBins];
    if (threadIdx.x < kNumBins) c[threadIdx.x] = 0;
    __syncthreads();
    int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r < nrows) atomicAdd(&c[bin_of_length(rp[r + 1] - rp[r])], 1);
    __syncthreads();
    if (threadIdx.x < kNumBins) cnt[(int64_t)threadIdx.x * nwg + blockIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int32_t nrows, const int32_t *rp,
                                                        const int32_t *off, int32_t nwg,
                                                        int32_t *list) {
    __shared__ int32_t wc[kBlock / kWave][kNumBins];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int b = r < nrows ? bin_of_length(rp[r + 1] - rp[r]) : -1;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    int my_rank = 0;
    for (int q = 0; q < kNumBins; ++q) {
        uint64_t m = __ballot(b == q);
        if (b == q) my_rank = __popcll(m & lt);
        if (lane == 0) wc[wave][q] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int32_t pos = off[(int64_t)b * nwg + blockIdx.x] + my_rank;
        for (int w = 0; w < wave; ++w) pos += wc[w][b];
        list[pos] = (int32_t)r;
    }
}

__global__ void k_bin_bounds(const int32_t *off, int32_t nwg, int32_t nrows, int32_t *bin_off) {
    int b = threadIdx.x;
    if (b < kNumBins) bin_off[b] = off[(int64_t)b * nwg];
    if (b == kNumBins) bin_off[b] = nrows;
}

// ---- gradient-based shuffle (Sections 5 and 8) -------------------------------------

__global__ __launch_bounds__(kBlock) void k_row_counts(int32_t nrows, const int32_t *rp,
                                                       int32_t *counts) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x)
        counts[i] = rp[i + 1] - rp[i];
}

__global__ __launch_bounds__(kBlock) void k_col_counts(int64_t nnz, const int32_t *col,
                                                       int32_t *counts) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&counts[col[e]], 1);
}

struct ArgMax { int64_t g; int64_t i; };

__device__ inline ArgMax better(ArgMax a, ArgMax b) {        // larger g; first index on ties
    return (b.g > a.g || (b.g == a.g && b.i < a.i)) ? b : a;
}

__device__ inline ArgMax block_argmax(ArgMax v, ArgMax *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = better(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    return sh[0];
}

// gradient g_i = h[i+1] - h[i], i < n - 1 (n >= 2)
__global__ __launch_bounds__(kBlock) void k_grad_argmax_partial(int64_t n, const int32_t *h,
                                                                ArgMax *part) {
    __shared__ ArgMax sh[kBlock];
    ArgMax best{INT64_MIN, INT64_MAX};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n - 1;
         i += (int64_t)gridDim.x * blockDim.x)
        best = better(best, ArgMax{(int64_t)h[i + 1] - h[i], i});
    best = block_argmax(best, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ __launch_bounds__(kBlock) void k_grad_argmax_final(int32_t nparts, const ArgMax *part,
                                                              int32_t *pivot) {
    __shared__ ArgMax sh[kBlock];
    ArgMax best{INT64_MIN, INT64_MAX};
    for (int i = threadIdx.x; i < nparts; i += kBlock) best = better(best, part[i]);
    best = block_argmax(best, sh);
    if (threadIdx.x == 0) *pivot = (int32_t)best.i;
}

// Riffle: A (local permutation pa of [0, na)) and B (pb of [0, nb), offset
// by na) alternate while both last; the longer part's remainder follows.
__global__ __launch_bounds__(kBlock) void k_riffle(int64_t na, int64_t nb, const int32_t *pa,
                                                   const int32_t *pb, int32_t *perm) {
    const int64_t m = na < nb ? na : nb, n = na + nb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t v;
        if (t < 2 * m) v = (t & 1) ? (int32_t)(na + pb[t >> 1]) : pa[t >> 1];
        else v = na > m ? pa[m + (t - 2 * m)] : (int32_t)(na + pb[m + (t - 2 * m)]);
        perm[t] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_invert(int64_t n, const int32_t *perm, int32_t *inv) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        inv[perm[k]] = (int32_t)k;
}

}  // namespace

// ============================ launchers ==========================================

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

size_t scan_ws_bytes(int64_t n) { return align256(sizeof(int32_t) * (size_t)(cdiv(n, kScanTile) + 1)); }

hipError_t launch_exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *ws,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t ntiles = cdiv(n, kScanTile);
    int32_t *sums = (int32_t *)ws;
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(ntiles), dim3(kBlock), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, sums, ntiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, s, in, out, n,
                       (const int32_t *)sums);
    return hipGetLastError();
}

size_t random_perm_ws_bytes(int64_t n) {
    if (n <= kLdsPermMax) {
        const int64_t nwg = std::max<int64_t>(1, cdiv(n, kPermItems));
        const int64_t ncounts = (nwg << radix_bits(n)) + 1;
        return align256(sizeof(int32_t) * ncounts) + align256(sizeof(int32_t) * (n + 1)) +
               scan_ws_bytes(ncounts);
    }
    int64_t nb = int64_t(1) << bucket_bits(n);
    return align256(sizeof(int32_t) * (nb + 1)) + 2 * align256(sizeof(int32_t) * (n + 1)) +
           scan_ws_bytes(nb + 1);
}

hipError_t launch_random_perm(int64_t n, uint64_t stream_seed, int32_t *perm, int32_t *inv,
                              void *ws, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n <= kLdsPermMax) {
        const int bits = radix_bits(n);
        const int32_t nd = 1 << bits;
        const int32_t nwg = (int32_t)std::max<int64_t>(1, cdiv(n, kPermItems));
        const int64_t ncounts = (int64_t)nwg * nd + 1;
        char *w = (char *)ws;
        int32_t *counts = (int32_t *)w;  w += align256(sizeof(int32_t) * ncounts);
        int32_t *items = (int32_t *)w;   w += align256(sizeof(int32_t) * (n + 1));
        void *scan_ws = w;
        const size_t lds = sizeof(int32_t) * (size_t)nd;
        hipLaunchKernelGGL(k_perm_count, dim3(nwg), dim3(kBlock), lds, s, n, stream_seed, bits, nwg,
                           counts);
        hipError_t e = launch_fill_i32(counts + ncounts - 1, 1, 0, s);
        if (e != hipSuccess) return e;
        if ((e = launch_exclusive_scan(counts, counts, ncounts, scan_ws, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_perm_scatter, dim3(nwg), dim3(kBlock), lds, s, n, stream_seed, bits, nwg,
                           (const int32_t *)counts, items);
        hipLaunchKernelGGL(k_perm_bucket_sort, dim3(nd), dim3(kBlock), 0, s, nd, nwg, stream_seed,
                           bits, (const int32_t *)counts, (const int32_t *)items, perm, inv);
        return hipGetLastError();
    }
    const int bits = bucket_bits(n);
    const int64_t nb = int64_t(1) << bits;
    char *w = (char *)ws;
    int32_t *counts = (int32_t *)w;  w += align256(sizeof(int32_t) * (nb + 1));
    int32_t *slot = (int32_t *)w;    w += align256(sizeof(int32_t) * (n + 1));
    int32_t *items = (int32_t *)w;   w += align256(sizeof(int32_t) * (n + 1));
    void *scan_ws = w;
    hipError_t e = launch_fill_i32(counts, nb + 1, 0, s);
    if (e != hipSuccess) return e;
    const int g = grid_for(n, kBlock, 8192);
    hipLaunchKernelGGL(k_bucket_count, dim3(g), dim3(kBlock), 0, s, n, stream_seed, bits, counts,
                       slot);
    e = launch_exclusive_scan(counts, counts, nb + 1, scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(g), dim3(kBlock), 0, s, n, stream_seed, bits,
                       (const int32_t *)counts, (const int32_t *)slot, items);
    hipLaunchKernelGGL(k_perm_bucket_sort, dim3((unsigned)nb), dim3(kBlock), 0, s, (int32_t)nb, 1,
                       stream_seed, bits, (const int32_t *)counts, (const int32_t *)items, perm, inv);
    return hipGetLastError();
}

size_t permuted_row_ptr_ws_bytes(int32_t nrows) { return scan_ws_bytes((int64_t)nrows + 1); }

hipError_t launch_permuted_row_ptr(int32_t nrows, const int32_t *rp, const int32_t *rperm,
                                   int32_t *rp_b, void *ws, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_row_len, dim3(grid_for((int64_t)nrows + 1, kBlock, 1 << 30)),
                       dim3(kBlock), 0, s, nrows, rp, rperm, rp_b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_exclusive_scan(rp_b, rp_b, (int64_t)nrows + 1, ws, s);
}

hipError_t launch_gather_relabel_sort(int32_t nrows, const int32_t *rp, const int32_t *col,
                                      const void *val, int val_bytes, const int32_t *rinv,
                                      const int32_t *cinv, const int32_t *rp_b, int32_t *col_b,
                                      void *val_b, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    const int64_t g = cdiv(nrows, (int64_t)kSortRows * kSortWaves);
    switch (val_bytes) {
    case 8:
        hipLaunchKernelGGL(k_gather_relabel_sort<uint64_t>, dim3((unsigned)g), dim3(kBlock), 0, s, nrows, rp,
                           col, (const uint64_t *)val, rinv, cinv, rp_b, col_b, (uint64_t *)val_b);
        break;
    case 4:
        hipLaunchKernelGGL(k_gather_relabel_sort<uint32_t>, dim3((unsigned)g), dim3(kBlock), 0, s, nrows, rp,
                           col, (const uint32_t *)val, rinv, cinv, rp_b, col_b, (uint32_t *)val_b);
        break;
    case 2:
        hipLaunchKernelGGL(k_gather_relabel_sort<uint16_t>, dim3((unsigned)g), dim3(kBlock), 0, s, nrows, rp,
                           col, (const uint16_t *)val, rinv, cinv, rp_b, col_b, (uint16_t *)val_b);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather_rows(int32_t n, int32_t k, const int32_t *perm, const void *X,
                              int64_t ldx, void *Xp, int64_t ldxp, int elem_bytes, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = grid_for(n, kBlock, 16384);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather_rows<double>, dim3(g), dim3(kBlock), 0, s, n, k, perm,
                           (const double *)X, ldx, (double *)Xp, ldxp);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_gather_rows<float>, dim3(g), dim3(kBlock), 0, s, n, k, perm,
                           (const float *)X, ldx, (float *)Xp, ldxp);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_scatter_rows(int32_t n, int32_t k, const int32_t *perm, const void *Yp,
                               int64_t ldyp, void *Y, int64_t ldy, int elem_bytes, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = grid_for(n, kBlock, 16384);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_scatter_rows<double>, dim3(g), dim3(kBlock), 0, s, n, k, perm,
                           (const double *)Yp, ldyp, (double *)Y, ldy);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_scatter_rows<float>, dim3(g), dim3(kBlock), 0, s, n, k, perm,
                           (const float *)Yp, ldyp, (float *)Y, ldy);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_copy_cols(int32_t n, int32_t k, const void *src, int64_t lds, void *dst,
                            int64_t ldd, int elem_bytes, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    const int g = grid_for(n, kBlock, 16384);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_copy_cols<double>, dim3(g), dim3(kBlock), 0, s, n, k,
                           (const double *)src, lds, (double *)dst, ldd);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_copy_cols<float>, dim3(g), dim3(kBlock), 0, s, n, k,
                           (const float *)src, lds, (float *)dst, ldd);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack_cols(const PackCols *table, int32_t count, int32_t max_n, int elem_bytes,
                            hipStream_t s) {
    if (count <= 0 || max_n <= 0) return hipSuccess;
    // max_n rows of up to 16 columns per entry
    const dim3 grid(grid_for((int64_t)max_n * 16, kBlock, 2048), count);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_pack_cols<double>, grid, dim3(kBlock), 0, s, table);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_pack_cols<float>, grid, dim3(kBlock), 0, s, table);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_convert_f64(const double *in, void *out, int64_t n, int dtype, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = grid_for(n, kBlock, 16384);
    if (dtype == VAL_F32)
        hipLaunchKernelGGL(k_f64_to_f32, dim3(g), dim3(kBlock), 0, s, in, (float *)out, n);
    else if (dtype == VAL_BF16)
        hipLaunchKernelGGL(k_f64_to_bf16, dim3(g), dim3(kBlock), 0, s, in, (uint16_t *)out, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_line_counts(bool rows, int32_t nrows, int64_t nnz, const int32_t *rp,
                              const int32_t *col, int32_t n, int32_t *counts, hipStream_t s) {
    if (rows) {
        if (nrows <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_row_counts, dim3(grid_for(nrows, kBlock, 16384)), dim3(kBlock), 0, s,
                           nrows, rp, counts);
        return hipGetLastError();
    }
    hipError_t e = launch_fill_i32(counts, n, 0, s);
    if (e != hipSuccess || nnz <= 0) return e;
    hipLaunchKernelGGL(k_col_counts, dim3(grid_for(nnz, kBlock, 16384)), dim3(kBlock), 0, s, nnz,
                       col, counts);
    return hipGetLastError();
}

namespace {
constexpr int kArgParts = 1024;
}

size_t gradient_perm_ws_bytes(int64_t n) {
    return align256(sizeof(ArgMax) * kArgParts) + 256 + align256(sizeof(int32_t) * (n + 1)) +
           random_perm_ws_bytes(n);
}

hipError_t launch_gradient_perm(int64_t n, const int32_t *counts, uint64_t stream_seed,
                                int32_t *perm, int32_t *inv, void *ws, hipStream_t s) {
    if (n < 2) {
        hipError_t e = launch_iota_i32(perm, n, s);
        return e != hipSuccess ? e : launch_iota_i32(inv, n, s);
    }
    char *w = (char *)ws;
    ArgMax *part = (ArgMax *)w;  w += align256(sizeof(ArgMax) * kArgParts);
    int32_t *pivot = (int32_t *)w;  w += 256;
    int32_t *pab = (int32_t *)w;  w += align256(sizeof(int32_t) * (n + 1));
    void *rws = w;
    const int g = grid_for(n - 1, kBlock, kArgParts);
    hipLaunchKernelGGL(k_grad_argmax_partial, dim3(g), dim3(kBlock), 0, s, n, counts, part);
    hipLaunchKernelGGL(k_grad_argmax_final, dim3(1), dim3(kBlock), 0, s, g, (const ArgMax *)part,
                       pivot);
    int32_t p = 0;
    hipError_t e = hipMemcpyAsync(&p, pivot, sizeof p, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);     // the pivot sizes the two parts
    if (e != hipSuccess) return e;
    const int64_t na = (int64_t)p + 1, nb = n - na;
    // part B's keys continue the stream at index na: key(s, na + i) = key(s + na*gamma, i)
    const uint64_t seed_b = stream_seed + (uint64_t)na * 0x9e3779b97f4a7c15ull;
    if ((e = launch_random_perm(na, stream_seed, pab, nullptr, rws, s)) != hipSuccess) return e;
    if ((e = launch_random_perm(nb, seed_b, pab + na, nullptr, rws, s)) != hipSuccess) return e;
    const int gr = grid_for(n, kBlock, 16384);
    hipLaunchKernelGGL(k_riffle, dim3(gr), dim3(kBlock), 0, s, na, nb, (const int32_t *)pab,
                       (const int32_t *)(pab + na), perm);
    hipLaunchKernelGGL(k_invert, dim3(gr), dim3(kBlock), 0, s, n, (const int32_t *)perm, inv);
    return hipGetLastError();
}

hipError_t launch_row_max(int32_t nrows, const int32_t *rp, int32_t *max_len, hipStream_t s) {
    hipError_t e = launch_fill_i32(max_len, 1, 0, s);
    if (e != hipSuccess || nrows <= 0) return e;
    hipLaunchKernelGGL(k_row_max, dim3(grid_for(nrows, kBlock, 2048)), dim3(kBlock), 0, s, nrows,
                       rp, max_len);
    return hipGetLastError();
}

size_t row_bins_ws_bytes(int32_t nrows) {
    int64_t nwg = cdiv(nrows, kBlock);
    int64_t n = kNumBins * nwg;
    return align256(sizeof(int32_t) * (n + 1)) + scan_ws_bytes(n);
}

hipError_t launch_row_bins(int32_t nrows, const int32_t *rp, int32_t *list, int32_t *bin_off,
                           void *ws, hipStream_t s) {
    const int32_t nwg = (int32_t)cdiv(nrows, kBlock);
    if (nrows <= 0) {
        hipError_t e = launch_fill_i32(bin_off, kNumBins + 1, 0, s);
        return e;
    }
    int32_t *cnt = (int32_t *)ws;
    void *scan_ws = (char *)ws + align256(sizeof(int32_t) * ((int64_t)kNumBins * nwg + 1));
    hipLaunchKernelGGL(k_bin_count, dim3(nwg), dim3(kBlock), 0, s, nrows, rp, cnt, nwg);
    hipError_t e = launch_exclusive_scan(cnt, cnt, (int64_t)kNumBins * nwg, scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scatter, dim3(nwg), dim3(kBlock), 0, s, nrows, rp,
                       (const int32_t *)cnt, nwg, list);
    hipLaunchKernelGGL(k_bin_bounds, dim3(1), dim3(kWave), 0, s, (const int32_t *)cnt, nwg, nrows,
                       bin_off);
    return hipGetLastError();
}

}  // namespace mxe
