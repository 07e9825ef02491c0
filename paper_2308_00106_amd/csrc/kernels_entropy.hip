// 2D block nonzero histogram and its Shannon entropy (Section 4, Eq.
// eq:entropy; Section 5's 2D histogram view) for gfx950.
//
// Histogram: one workgroup per block-row (split further only when a block-row
// holds more than 64K entries). The block-row's entries are a contiguous
// nonzero range [row_ptr[r0], row_ptr[r1]), so the workgroup streams col_idx
// once, coalesced, and counts into an LDS copy of its G_c bins. Runs of equal
// block-column among neighbouring lanes (common in clustered matrices, whose
// sorted columns fall in the same block) are merged with one LDS atomic per
// run. A workgroup that owns its block-row writes the bins with plain stores.
//
// Entropy: H = ln S - (1/S) sum_b h_b ln h_b (nats), the same real number as
// -sum p ln p with p = h / S. Every term is evaluated in double-double (about
// 106 bits) with a fixed reduction order, so the result is deterministic; the
// final rounding to FP64 is certified against an error bound, which makes it
// the correctly rounded value of the exact entropy.
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <vector>

namespace mxe {

namespace {

constexpr int kBlock = 256;
constexpr int kHistLds = 16384;                 // block-columns held in LDS (at most 64 KB)
constexpr int64_t kHistSplitItems = 16384;      // entries per workgroup before splitting
constexpr int64_t kHistMinGroups = 2048;        // workgroups enough to fill the chip
constexpr int kEntGrid = 1024;                  // fixed grid: fixed reduction order

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// grid: (grid_r, split). Block-row bi covers rows [ceil(bi M / G_r), ceil((bi+1) M / G_r)).
__global__ __launch_bounds__(kBlock) void k_block_hist(int32_t nrows, int32_t ncols,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       int32_t grid_r, int32_t grid_c,
                                                       double inv_n, uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t bins[];                  // grid_c counters when they fit
    const int64_t bi = blockIdx.x;
    const int split = gridDim.y, part = blockIdx.y;
    const int64_t r0 = (bi * nrows + grid_r - 1) / grid_r;
    const int64_t r1 = ((bi + 1) * nrows + grid_r - 1) / grid_r;
    const int64_t e0 = rp[r0], e1 = rp[r1];
    const int64_t len = e1 - e0;
    const int64_t a = e0 + len * part / split, b = e0 + len * (part + 1) / split;
    const bool in_lds = grid_c <= kHistLds;
    uint32_t *out_row = hist + bi * grid_c;
    if (in_lds) {
        for (int c = threadIdx.x; c < grid_c; c += kBlock) bins[c] = 0;
        __syncthreads();
    }
    const int lane = threadIdx.x & (kWave - 1);
    // the workgroup walks [a, b) in steps of kBlock, so every wave is either
    // fully inside or partly inside a step: loop bounds are uniform per wave
    for (int64_t base = a; base < b; base += kBlock) {
        const int64_t e = base + threadIdx.x;
        const bool valid = e < b;
        const int32_t bj = valid ? block_index(col[e], grid_c, ncols, inv_n) : -1;
        if (in_lds) {
            const int32_t prev = __shfl_up(bj, 1);
            const bool head = valid && (lane == 0 || prev != bj);
            const uint64_t heads = __ballot(head);
            const uint64_t live = __ballot(valid);
            if (head) {
                const uint64_t above = lane == kWave - 1 ? 0ull : heads & (~0ull << (lane + 1));
                const int end = above ? __builtin_ctzll(above) : 64 - __builtin_clzll(live);
                atomicAdd(&bins[bj], (uint32_t)(end - lane));
            }
        } else if (valid) {
            atomicAdd(&out_row[bj], 1u);
        }
    }
    if (in_lds) {
        __syncthreads();
        if (split == 1) {
            for (int c = threadIdx.x; c < grid_c; c += kBlock) out_row[c] = bins[c];
        } else {
            for (int c = threadIdx.x; c < grid_c; c += kBlock)
                if (bins[c]) atomicAdd(&out_row[c], bins[c]);
        }
    }
}

// 2 atanh(u) = ln((1 + u) / (1 - u)) by its odd power series, |u| <= 0.2.
__device__ inline dd dd_two_atanh(dd u, const dd *coef) {
    dd w = dd_mul(u, u);
    dd acc = coef[kLnTerms - 1];
    for (int k = kLnTerms - 2; k >= 0; --k) acc = dd_add(dd_mul(acc, w), coef[k]);
    dd r = dd_mul(u, acc);
    return dd{2.0 * r.hi, 2.0 * r.lo};
}

// coef[k] = 1/(2k+1) and ln 2 = 4 atanh(1/7) + 2 atanh(1/17), i.e.
// ln 2 = 2 ln(4/3) + ln(9/8), set up in LDS by each workgroup.
__device__ inline void setup_log_tables(dd *coef, dd *ln2) {
    if (threadIdx.x < kLnTerms)
        coef[threadIdx.x] = dd_div(dd{1.0, 0.0}, dd{2.0 * threadIdx.x + 1.0, 0.0});
    __syncthreads();
    if (threadIdx.x == 0) {
        dd a = dd_two_atanh(dd_div(dd{1.0, 0.0}, dd{7.0, 0.0}), coef);
        dd b = dd_two_atanh(dd_div(dd{1.0, 0.0}, dd{17.0, 0.0}), coef);
        *ln2 = dd_add(dd{2.0 * a.hi, 2.0 * a.lo}, b);
    }
    __syncthreads();
}

struct EntPartial { double hi, lo; unsigned long long s, nz; };

__device__ inline void block_reduce(dd &acc, unsigned long long &s, unsigned long long &nz,
                                    dd *sh, unsigned long long *ss, unsigned long long *sz) {
    sh[threadIdx.x] = acc;
    ss[threadIdx.x] = s;
    sz[threadIdx.x] = nz;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[threadIdx.x] = dd_add(sh[threadIdx.x], sh[threadIdx.x + w]);
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sz[threadIdx.x] += sz[threadIdx.x + w];
        }
        __syncthreads();
    }
    acc = sh[0];
    s = ss[0];
    nz = sz[0];
}

// Count of counts: cc[c] = number of bins holding exactly c entries, for
// c < kCountDirect (LDS per workgroup, then exact integer atomics into one
// table); bins with more entries add c ln c to the workgroup's partial
// directly. S and the nonzero-bin count are summed alongside.
constexpr int kCountDirect = 4096;

__global__ __launch_bounds__(kBlock) void k_entropy_counts(const uint32_t *__restrict__ hist,
                                                           int64_t bins, uint32_t *__restrict__ cc,
                                                           EntPartial *part) {
    __shared__ uint32_t lcc[kCountDirect];
    __shared__ dd coef[kLnTerms];
    __shared__ dd ln2;
    __shared__ dd sh[kBlock];
    __shared__ unsigned long long ss[kBlock], sz[kBlock];
    for (int c = threadIdx.x; c < kCountDirect; c += kBlock) lcc[c] = 0;
    setup_log_tables(coef, &ln2);                         // synchronizes
    dd acc{0.0, 0.0};
    unsigned long long s = 0, nz = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < bins;
         i += (int64_t)gridDim.x * kBlock) {
        const uint32_t h = hist[i];
        s += h;
        nz += h != 0;
        if (h < kCountDirect) {
            if (h >= 2) atomicAdd(&lcc[h], 1u);
        } else {
            const double hd = (double)h;
            acc = dd_add(acc, dd_mul_d(dd_ln_int(hd, ln2, coef), hd));
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kCountDirect; c += kBlock)
        if (lcc[c]) atomicAdd(&cc[c], lcc[c]);
    block_reduce(acc, s, nz, sh, ss, sz);
    if (threadIdx.x == 0) part[blockIdx.x] = EntPartial{acc.hi, acc.lo, s, nz};
}

// Rounds v (absolute error <= eps) to FP64; *ok = 0 when v - eps and v + eps
// round differently (the correctly rounded value is then not certain).
__device__ inline double certified_round(dd v, double eps, int *ok) {
    double lo = v.hi + (v.lo - eps);
    double hi = v.hi + (v.lo + eps);
    if (lo != hi) *ok = 0;
    return v.hi + v.lo;
}

// From T = sum h ln h (double-double), S = sum h and the count of nonzero
// bins: result = {H bits, H nats, certified (1/0), S}, each H rounded to FP64
// and certified against the error bound (Eq. 2 with p = h / S).
__device__ inline void entropy_finish(dd acc, unsigned long long s, unsigned long long nz, dd ln2,
                                      const dd *coef, double *result) {
    if (s == 0 || nz <= 1) {            // no distribution, or all mass in one bin
        result[0] = 0.0;
        result[1] = 0.0;
        result[2] = 1.0;
        result[3] = (double)s;
        return;
    }
    const double sd = (double)s;        // exact: s < 2^53
    dd ln_s = dd_ln_int(sd, ln2, coef);
    dd mean = dd_div(acc, dd{sd, 0.0});
    dd h_nats = dd_sub(ln_s, mean);
    dd h_bits = dd_div(h_nats, ln2);
    // error bound: every double-double step is accurate to ~2^-100 relative and
    // the reduction is ~30 levels deep; 2^-90 (ln S + 1) leaves a 2^7 margin
    const double eps = 0x1p-90 * (ln_s.hi + 1.0);
    int ok = 1;
    result[0] = certified_round(h_bits, eps * 2.0, &ok);
    result[1] = certified_round(h_nats, eps, &ok);
    result[2] = ok ? 1.0 : 0.0;
    result[3] = sd;
}

// T = sum over c of cc[c] c ln c (c in fixed order per thread, then a fixed
// tree) plus the large-count partials in workgroup order.
__global__ __launch_bounds__(kBlock) void k_entropy_final(const uint32_t *__restrict__ cc,
                                                          const EntPartial *part, int nparts,
                                                          double *result) {
    __shared__ dd coef[kLnTerms];
    __shared__ dd ln2;
    __shared__ dd sh[kBlock];
    __shared__ unsigned long long ss[kBlock], sz[kBlock];
    setup_log_tables(coef, &ln2);
    dd acc{0.0, 0.0};
    unsigned long long s = 0, nz = 0;
    for (int c = 2 + threadIdx.x; c < kCountDirect; c += kBlock) {
        if (cc[c] == 0) continue;
        const double cd = (double)c;
        acc = dd_add(acc, dd_mul_d(dd_mul_d(dd_ln_int(cd, ln2, coef), cd), (double)cc[c]));
    }
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        acc = dd_add(acc, dd{part[i].hi, part[i].lo});
        s += part[i].s;
        nz += part[i].nz;
    }
    block_reduce(acc, s, nz, sh, ss, sz);
    if (threadIdx.x == 0) entropy_finish(acc, s, nz, ln2, coef, result);
}

// Hierarchical 2D entropy (Section 5). Region r covers bins [r0, r1) x
// [c0, c1) of the grid; `parts` workgroups share each region, workgroup p
// taking cells p*kBlock + t, p*kBlock + t + parts*kBlock, ... of it, and one
// workgroup per region then combines the parts in index order.
struct Region { int32_t r0, r1, c0, c1; };

__global__ __launch_bounds__(kBlock) void k_entropy_regions_partial(
    const uint32_t *__restrict__ hist, int32_t grid_c, const Region *__restrict__ regions,
    int32_t parts, EntPartial *__restrict__ part) {
    __shared__ dd coef[kLnTerms];
    __shared__ dd ln2;
    __shared__ dd sh[kBlock];
    __shared__ unsigned long long ss[kBlock], sz[kBlock];
    setup_log_tables(coef, &ln2);
    const int64_t region = blockIdx.x / parts, p = blockIdx.x % parts;
    const Region rg = regions[region];
    const int64_t w = rg.c1 - rg.c0, cells = (int64_t)(rg.r1 - rg.r0) * w;
    dd acc{0.0, 0.0};
    unsigned long long s = 0, nz = 0;
    for (int64_t i = p * kBlock + threadIdx.x; i < cells; i += (int64_t)parts * kBlock) {
        const uint32_t h = hist[(int64_t)(rg.r0 + i / w) * grid_c + rg.c0 + i % w];
        s += h;
        nz += h != 0;
        if (h >= 2) {
            const double hd = (double)h;
            acc = dd_add(acc, dd_mul_d(dd_ln_int(hd, ln2, coef), hd));
        }
    }
    block_reduce(acc, s, nz, sh, ss, sz);
    if (threadIdx.x == 0) part[blockIdx.x] = EntPartial{acc.hi, acc.lo, s, nz};
}

__global__ __launch_bounds__(kBlock) void k_entropy_regions_final(const EntPartial *__restrict__ part,
                                                                  int32_t parts,
                                                                  double *__restrict__ out) {
    __shared__ dd coef[kLnTerms];
    __shared__ dd ln2;
    __shared__ dd sh[kBlock];
    __shared__ unsigned long long ss[kBlock], sz[kBlock];
    setup_log_tables(coef, &ln2);
    const EntPartial *pr = part + (int64_t)blockIdx.x * parts;
    dd acc{0.0, 0.0};
    unsigned long long s = 0, nz = 0;
    for (int i = threadIdx.x; i < parts; i += kBlock) {
        acc = dd_add(acc, dd{pr[i].hi, pr[i].lo});
        s += pr[i].s;
        nz += pr[i].nz;
    }
    block_reduce(acc, s, nz, sh, ss, sz);
    if (threadIdx.x == 0) entropy_finish(acc, s, nz, ln2, coef, out + 4 * (int64_t)blockIdx.x);
}

// Workgroups per region: enough that the largest region's cells are spread
// at ~16 per thread, at most 64, and about 16K workgroups in total.
int32_t region_parts(int32_t grid_r, int32_t grid_c, const int32_t *levels, int32_t nlevels,
                     int32_t nregions) {
    int64_t max_cells = 0;
    for (int32_t i = 0; i < nlevels; ++i) {
        const int64_t lr = std::min(levels[i], grid_r), lc = std::min(levels[i], grid_c);
        max_cells = std::max(max_cells, cdiv(grid_r, lr) * cdiv(grid_c, lc));
    }
    int64_t p = cdiv(max_cells, 16 * (int64_t)kBlock);
    p = std::min<int64_t>(p, 64);
    p = std::min<int64_t>(p, std::max<int64_t>(1, 16384 / std::max(nregions, 1)));
    return (int32_t)std::max<int64_t>(p, 1);
}

}  // namespace

hipError_t launch_block_hist(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rp,
                             const int32_t *col, int32_t grid_r, int32_t grid_c, uint32_t *hist,
                             hipStream_t s) {
    const int64_t bins = (int64_t)grid_r * grid_c;
    int64_t split = std::max(cdiv(cdiv(nnz, grid_r), kHistSplitItems), cdiv(kHistMinGroups, grid_r));
    if (split < 1) split = 1;
    if (split > 65535) split = 65535;
    const bool needs_zero = split > 1 || grid_c > kHistLds;
    if (needs_zero) {
        int g = (int)std::min<int64_t>(cdiv(bins, kBlock), 65536);
        hipLaunchKernelGGL(k_zero_u32, dim3(g), dim3(kBlock), 0, s, hist, bins);
    }
    const double inv_n = 1.0 / (double)ncols;
    const size_t lds = grid_c <= kHistLds ? sizeof(uint32_t) * (size_t)grid_c : 0;
    hipLaunchKernelGGL(k_block_hist, dim3(grid_r, (unsigned)split), dim3(kBlock), lds, s, nrows,
                       ncols, rp, col, grid_r, grid_c, inv_n, hist);
    return hipGetLastError();
}

size_t entropy_ws_bytes(int64_t) {
    return sizeof(uint32_t) * kCountDirect + sizeof(EntPartial) * kEntGrid + 256;
}

hipError_t launch_entropy(const uint32_t *hist, int64_t bins, double *result, void *ws,
                          hipStream_t s) {
    uint32_t *cc = (uint32_t *)ws;
    EntPartial *part = (EntPartial *)(cc + kCountDirect);
    hipLaunchKernelGGL(k_zero_u32, dim3(kCountDirect / kBlock), dim3(kBlock), 0, s, cc,
                       (int64_t)kCountDirect);
    int g = (int)std::min<int64_t>(kEntGrid, std::max<int64_t>(1, cdiv(bins, kBlock)));
    hipLaunchKernelGGL(k_entropy_counts, dim3(g), dim3(kBlock), 0, s, hist, bins, cc, part);
    hipLaunchKernelGGL(k_entropy_final, dim3(1), dim3(kBlock), 0, s, (const uint32_t *)cc,
                       (const EntPartial *)part, g, result);
    return hipGetLastError();
}

int32_t entropy_regions_count(int32_t grid_r, int32_t grid_c, const int32_t *levels,
                              int32_t nlevels) {
    int32_t n = 0;
    for (int32_t i = 0; i < nlevels; ++i)
        n += std::min(levels[i], grid_r) * std::min(levels[i], grid_c);
    return n;
}

size_t entropy_regions_ws_bytes(int32_t grid_r, int32_t grid_c, const int32_t *levels,
                                int32_t nlevels) {
    const int32_t n = entropy_regions_count(grid_r, grid_c, levels, nlevels);
    const int64_t parts = region_parts(grid_r, grid_c, levels, nlevels, n);
    return ((sizeof(Region) * (size_t)n + 255) & ~size_t(255)) +
           sizeof(EntPartial) * (size_t)n * (size_t)parts;
}

hipError_t launch_entropy_regions(const uint32_t *hist, int32_t grid_r, int32_t grid_c,
                                  const int32_t *levels, int32_t nlevels, double *result,
                                  void *ws, hipStream_t s) {
    // region (a, b) of level L holds the bins r with floor(r * Lr / G_r) = a,
    // i.e. r in [ceil(a G_r / Lr), ceil((a + 1) G_r / Lr)), and likewise columns
    std::vector<Region> regs;
    for (int32_t i = 0; i < nlevels; ++i) {
        const int64_t lr = std::min(levels[i], grid_r), lc = std::min(levels[i], grid_c);
        for (int64_t a = 0; a < lr; ++a)
            for (int64_t b = 0; b < lc; ++b)
                regs.push_back(Region{(int32_t)((a * grid_r + lr - 1) / lr),
                                      (int32_t)(((a + 1) * grid_r + lr - 1) / lr),
                                      (int32_t)((b * grid_c + lc - 1) / lc),
                                      (int32_t)(((b + 1) * grid_c + lc - 1) / lc)});
    }
    if (regs.empty()) return hipSuccess;
    const int32_t n = (int32_t)regs.size();
    const int32_t parts = region_parts(grid_r, grid_c, levels, nlevels, n);
    Region *dregs = (Region *)ws;
    EntPartial *part = (EntPartial *)((char *)ws + ((sizeof(Region) * (size_t)n + 255) & ~size_t(255)));
    hipError_t e = hipMemcpyAsync(dregs, regs.data(), sizeof(Region) * regs.size(),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    // the staging copy must land before the host vector goes away
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_entropy_regions_partial, dim3((unsigned)((int64_t)n * parts)), dim3(kBlock),
                       0, s, hist, grid_c, (const Region *)dregs, parts, part);
    hipLaunchKernelGGL(k_entropy_regions_final, dim3((unsigned)n), dim3(kBlock), 0, s,
                       (const EntPartial *)part, parts, result);
    return hipGetLastError();
}

}  // namespace mxe
