// Row-oriented CSR product helpers shared by the SpMV kernels
// (kernels_spmv.hip) and the persistent batch kernel (kernels_batch.hip).
#pragma once

#include "device_common.h"
#include "internal.h"

namespace mxe {

// val / col / row_ptr are streamed once: non-temporal loads keep them from
// evicting the gathered x lines.
template <typename P>
__device__ inline P ld_stream(const P *p) { return __builtin_nontemporal_load(p); }

template <typename V, typename T> struct ValLoad;
template <> struct ValLoad<double, double> {
    __device__ static double get(const double *p) { return ld_stream(p); }
};
template <> struct ValLoad<float, float> {
    __device__ static float get(const float *p) { return ld_stream(p); }
};
template <> struct ValLoad<uint16_t, float> {
    __device__ static float get(const uint16_t *p) { return bf16_to_f32(ld_stream(p)); }
};

// Rows [r0, r1) by a workgroup of NT threads (tid: the thread's index), with
// the lane count L and column count KM as runtime values (KM = the k class,
// L >= KM, both powers of two dividing 64): groups of L lanes take one row at
// a time, KM column lanes times L / KM entry lanes, then an xor butterfly over
// the entry lanes. One code path for every (L, KM) keeps a single accumulator
// in registers. Groups are L-aligned, so the shuffles stay inside a group.
// ycol (may be null): column q of the result goes to ycol[q] (its row 0) with
// leading dimension ycol_ld[q] instead of Y + q with ldy.
template <typename V, typename T, int NT>
__device__ inline void rows_runtime(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                    const V *__restrict__ val, int32_t k, const T *__restrict__ X,
                                    int64_t ldx, T *__restrict__ Y, int64_t ldy, int L, int KM,
                                    int32_t r0, int32_t r1, int tid, void *const *ycol = nullptr,
                                    const int64_t *ycol_ld = nullptr) {
    const int E = L / KM;
    const int lane = tid % L, q = lane % KM, el = lane / KM;
    const bool active = q < k;
    for (int32_t row = r0 + tid / L; row < r1; row += NT / L) {
        const int32_t s = ld_stream(rp + row), e = ld_stream(rp + row + 1);
        T acc = T(0);
        int32_t p = s + el;
        for (; p + E < e; p += 2 * E) {
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
        for (int off = L / 2; off >= KM; off >>= 1) acc += __shfl_xor(acc, off);
        if (el == 0 && active) {
            if (ycol) as_global(static_cast<T *>(ycol[q]))[(int64_t)row * ycol_ld[q]] = acc;
            else Y[(int64_t)row * ldy + q] = acc;
        }
    }
}

}  // namespace mxe
