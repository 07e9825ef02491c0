// The column-slab product of one workgroup block, shared by the slab SpMV
// kernel (one block per workgroup) and the persistent batch kernel (blocks of
// many matrices pulled from per-XCD queues). Layout and geometry: SlabGeom in
// internal.h, built by kernels_slab.hip.
#pragma once

#include "device_common.h"
#include "internal.h"

namespace mxe {

constexpr int kSlabBlock = 1024;                    // 16 wavefronts
constexpr int kSubBlocks = kSlabBlock / kWave;      // wavefront sub-blocks per block
constexpr int kSlabMax = 64;                        // column slabs per layout
// 64-entry chunks each wavefront keeps in flight. IF = 0 (the single-product
// kernels): four for one or two right-hand sides, two for four, one above.
// IF > 0 (the persistent batch kernel): as many as keep about IF bytes of x
// per lane in flight, 1 to 8.
template <int KM, typename T, int IF> struct SlabUnroll {
    static constexpr int B = IF / (KM * (int)sizeof(T));
    static constexpr int value = IF == 0 ? (KM <= 2 ? 4 : KM <= 4 ? 2 : 1) : B < 1 ? 1 : B > 8 ? 8 : B;
};
template <typename V, typename T> struct SlabVal;
template <> struct SlabVal<double, double> {
    __device__ static double get(double v) { return v; }
};
template <> struct SlabVal<float, float> {
    __device__ static float get(float v) { return v; }
};
template <> struct SlabVal<uint16_t, float> {
    __device__ static float get(uint16_t v) { return bf16_to_f32(v); }
};

// Block `block` of the layout, by a workgroup of kSlabBlock threads; tid is
// the thread's index in it. The workgroup walks the slabs in a rotation that
// starts at the slab tied to XCD `xcd` (its own XCD; in a batch, the XCD of
// the queue the block came from), all together (a barrier after each slab),
// so its wavefronts gather from the same L2-resident x slice; inside a slab a
// wavefront loads up to SlabUnroll<KM, T, IF> chunks of its group at once, issues their x
// gathers together, then reduces each chunk by row. The first batch of the
// next slab's group is loaded before each barrier. yp: LDS for the block's
// partial y (rows_per_block x KM values of T); soff: LDS for the wavefronts'
// group offsets; vec_x: X rows are read as vectors of min(16, KM x sizeof(T))
// bytes (slab_vec_x). The
// caller separates two calls on one workgroup by a barrier.
// WIN: X rows [w0, w0 + win) are first copied to LDS (xw, win x KM values of
// T), and entries whose column falls there read x from LDS instead of
// gathering it (the same values, so the same sums).
// ycol (may be null): column q of the result goes to ycol[q] (its row 0)
// with leading dimension ycol_ld[q] instead of Y + q with ldy.
// prio (one right-hand side): the wavefront raises its issue priority while
// it sends out a batch's x gathers and drops it for the reductions.
template <typename V, typename T, int KM, int SR, bool WIN = false, int IF = 0>
__device__ __attribute__((always_inline)) inline void
slab_block(const SlabGeom &g, int32_t block, int xcd, const int32_t *__restrict__ off,
           const uint32_t *__restrict__ idx, const V *__restrict__ val, int32_t k,
           const T *__restrict__ X, int64_t ldx, T *__restrict__ Y, int64_t ldy, int vec_x,
           T *yp, int32_t (*soff)[kSlabMax + 1], int tid, T *xw = nullptr, int32_t w0 = 0,
           int32_t win = 0, void *const *ycol = nullptr, const int64_t *ycol_ld = nullptr,
           bool prio = false) {
    using S = Semiring<SR, T>;
    const int wave = tid / kWave, lane = tid % kWave;
    const int32_t R = g.rows_per_block;
    for (int i = tid; i < R * KM; i += kSlabBlock) yp[i] = S::identity();
    if constexpr (WIN) {
        for (int32_t i = tid; i < win * KM; i += kSlabBlock) {
            const int32_t r = w0 + i / KM, q = i % KM;
            xw[i] = (r < g.ncols && (KM == 1 || q < k)) ? X[(int64_t)r * ldx + q] : T(0);
        }
    }
    T *ywave = yp + (int64_t)wave * g.rows_per_sub * KM;
    // this wavefront's groups (one per slab) and their offsets
    const int32_t *o = off + ((int64_t)block * kSubBlocks + wave) * g.slabs;
    for (int s = lane; s <= g.slabs; s += kWave) soff[wave][s] = o[s];
    __syncthreads();
    const int s0 = (int)(((int64_t)xcd * g.slabs) / 8);
    const uint32_t cmask = (1u << g.cbits) - 1u;
    constexpr int kD = SlabUnroll<KM, T, IF>::value;
    uint32_t u[kD];
    // values as stored, widened where they are used: widening BF16 here, in
    // the branch that loads it, made each chunk wait for its value before the
    // next chunk's loads went out
    V a[kD];
    auto load_batch = [&](int32_t c, int32_t e) {             // up to kD chunks of [c, e)
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            const int32_t p = c + j * kWave + lane;
            const bool v = p < e;
            u[j] = v ? idx[p] : 0xffffffffu;
            a[j] = v ? val[p] : V{};
        }
    };
    load_batch(soff[wave][s0], soff[wave][s0 + 1]);
    for (int t = 0; t < g.slabs; ++t) {                       // same count in every wavefront
        const int s = s0 + t < g.slabs ? s0 + t : s0 + t - g.slabs;
        const int32_t b = soff[wave][s], e = soff[wave][s + 1];
        for (int32_t c = b; c < e; c += kD * kWave) {
            if (c != b) load_batch(c, e);                     // the first batch is already loaded
            T xv[kD][KM];
            if constexpr (KM == 1) {
                if (prio) __builtin_amdgcn_s_setprio(2);
            }
#pragma unroll
            for (int j = 0; j < kD; ++j) {
                const bool v = u[j] != 0xffffffffu;
                if constexpr (WIN) {
                    const uint32_t d = (u[j] & cmask) - (uint32_t)w0;
                    if (v && d < (uint32_t)win) {
#pragma unroll
                        for (int q = 0; q < KM; ++q) xv[j][q] = xw[(int64_t)d * KM + q];
                        continue;
                    }
                }
                const T *xr = X + (int64_t)(v ? (u[j] & cmask) : 0) * ldx;
                if constexpr (KM > 1) {
                    if (vec_x) {                              // k == KM, rows aligned to the vector
                        constexpr int W = (16 / (int)sizeof(T)) < KM ? 16 / (int)sizeof(T) : KM;
                        typedef T vec_t __attribute__((ext_vector_type(W)));
#pragma unroll
                        for (int q = 0; q < KM; q += W) {
                            const vec_t w = *reinterpret_cast<const vec_t *>(xr + q);
#pragma unroll
                            for (int r = 0; r < W; ++r) xv[j][q + r] = v ? w[r] : T(0);
                        }
                        continue;
                    }
                }
#pragma unroll
                for (int q = 0; q < KM; ++q) xv[j][q] = (v && (KM == 1 || q < k)) ? xr[q] : T(0);
            }
            if constexpr (KM == 1) {
                if (prio) __builtin_amdgcn_s_setprio(0);
            }
#pragma unroll
            for (int j = 0; j < kD; ++j) {
                if (c + j * kWave >= e) break;                // uniform per wavefront
                // padding lanes (key 0xffffffff) sit after every valid lane
                const uint32_t key = u[j] != 0xffffffffu ? (u[j] >> g.cbits) : 0xffffffffu;
                const T aj = SlabVal<V, T>::get(a[j]);
                T prod[KM];
#pragma unroll
                for (int q = 0; q < KM; ++q) prod[q] = S::mul(aj, xv[j][q]);
                if constexpr (SR == 0) segmented_scan<T, KM>(key, prod);
                else segmented_scan_op<S, T, KM>(key, prod);
                const uint32_t nxt = __shfl_down(key, 1);
                const bool tail = key != 0xffffffffu && (lane == kWave - 1 || nxt != key);
                if (tail) {
#pragma unroll
                    for (int q = 0; q < KM; ++q)
                        ywave[(int64_t)key * KM + q] = S::add(ywave[(int64_t)key * KM + q], prod[q]);
                }
                // the next chunk's tails may update the same rows: keep order
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (t + 1 < g.slabs) {                                // next slab's first batch, issued
            const int sn = s + 1 < g.slabs ? s + 1 : 0;       // before the barrier waits
            load_batch(soff[wave][sn], soff[wave][sn + 1]);
        }
        __syncthreads();
    }
    const int64_t row0 = (int64_t)block * R;
    for (int i = tid; i < R * KM; i += kSlabBlock) {
        const int64_t row = row0 + i / KM;
        const int q = i % KM;
        if (row < g.nrows && (KM == 1 || q < k)) {
            // y is streamed out: non-temporal stores leave no dirty lines in
            // the L2 for the end of the launch to write back
            if (ycol) __builtin_nontemporal_store(yp[i], &as_global(static_cast<T *>(ycol[q]))[row * ycol_ld[q]]);
            else __builtin_nontemporal_store(yp[i], &Y[row * ldy + q]);
        }
    }
}

}  // namespace mxe
