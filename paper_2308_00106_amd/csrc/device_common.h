// Device helpers shared by the mxe kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxe {

constexpr int kWave = 64;

// A pointer the caller knows to address device memory, in a form the compiler
// can prove it of. Pointers read from memory (a batch's descriptors) are
// otherwise generic, and accesses through them compile to flat instructions,
// which also count against the LDS wait counter: every LDS wait then waits
// for all loads in flight as well.
template <typename T>
__device__ __attribute__((always_inline)) inline T *as_global(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// ---------------------------------------------------------------------------
// Random keys. The permutation of n items is the stable ascending order of
// key(s, i), the i-th output (i = 0, 1, ...) of SplitMix64 started at state s
// (Steele, Lea and Flood, OOPSLA 2014). SplitMix64 advances its state by the
// golden-ratio increment before each output, so output i is the finaliser
// applied to s + (i + 1) * increment: a counter-based hash, computed per index
// with no state and no memory traffic.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t sm64_key(uint64_t s, uint64_t i) {
    uint64_t z = s + (i + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Exact block index floor(j * g / n) for 0 <= j < n < 2^31, 1 <= g <= 2^20
// (the product stays below 2^51, exact in FP64). The FP64 quotient is within
// one of the true floor; one integer correction step makes it exact.
// ---------------------------------------------------------------------------
__device__ inline int32_t block_index(int64_t j, int64_t g, int64_t n, double inv_n) {
    int64_t num = j * g;
    int64_t q = (int64_t)((double)num * inv_n);
    if (q * n > num) --q;
    else if ((q + 1) * n <= num) ++q;
    return (int32_t)q;
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (about 106 significant bits), built from the
// error-free transformations of Knuth (two-sum) and the exact FMA product.
// Used to evaluate the entropy accurately enough to certify its rounding.
// ---------------------------------------------------------------------------
struct dd { double hi, lo; };

#pragma clang fp contract(off)
__device__ inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ inline dd quick_two_sum(double a, double b) {   // |a| >= |b|
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__device__ inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = __builtin_fma(a, b, -p);
    return {p, e};
}
__device__ inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ inline dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo;
    p.lo += a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_div(dd a, dd b) {
    // long division: two quotient digits and a correction
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}
#pragma clang fp contract(on)

// ln(m) for m in [sqrt(1/2), sqrt(2)]: 2 atanh(u), u = (m - 1) / (m + 1),
// |u| <= 0.1716, summed as u * sum_k u^(2k) / (2k + 1) for k < 24; u^2 < 2^-5.08,
// so the truncated tail is below 2^-120 of the sum. coef[k] = 1 / (2k + 1) in double-double.
constexpr int kLnTerms = 24;

__device__ inline dd dd_ln_reduced(dd m, const dd *coef) {
    dd num = dd_sub(m, dd{1.0, 0.0});
    dd den = dd_add(m, dd{1.0, 0.0});
    dd u = dd_div(num, den);
    dd w = dd_mul(u, u);
    dd acc = coef[kLnTerms - 1];
    for (int k = kLnTerms - 2; k >= 0; --k) acc = dd_add(dd_mul(acc, w), coef[k]);
    dd r = dd_mul(u, acc);
    return dd{2.0 * r.hi, 2.0 * r.lo};
}

// ln(x) for an integer-valued double 1 <= x < 2^53: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), then ln x = e ln2 + ln m (ln2 passed in).
__device__ inline dd dd_ln_int(double x, dd ln2, const dd *coef) {
    int e;
    double m = __builtin_frexp(x, &e);        // x = m 2^e, m in [0.5, 1)
    m *= 2.0;
    e -= 1;                                   // m in [1, 2)
    if (m > 1.4142135623730951) { m *= 0.5; e += 1; }
    dd lm = dd_ln_reduced(dd{m, 0.0}, coef);
    return dd_add(dd_mul_d(ln2, (double)e), lm);
}

// ---------------------------------------------------------------------------
// Value storage conversions, round to nearest, ties to even, from FP64.
// ---------------------------------------------------------------------------
__device__ inline uint16_t bf16_from_f64(double d) {
    uint64_t u = __double_as_longlong(d);
    uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
    uint64_t a = u & 0x7fffffffffffffffull;
    if (a > 0x7ff0000000000000ull) return sign | 0x7fc0u;          // NaN
    if (a == 0x7ff0000000000000ull) return sign | 0x7f80u;         // infinity
    int e = (int)(a >> 52) - 1023;                                 // unbiased exponent
    if (e < -134) return sign;                                     // below half the least subnormal
    uint64_t m = (a & 0x000fffffffffffffull) | 0x0010000000000000ull;  // value = m 2^(e-52)
    int qexp = e >= -126 ? e - 7 : -133;                           // BF16 spacing at this value
    int shift = qexp - (e - 52);                                   // 45 .. 53
    uint64_t kept = m >> shift;
    uint64_t rem = m & ((1ull << shift) - 1);
    uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (kept & 1))) ++kept;
    if (qexp == -133) return sign | (uint16_t)kept;                // subnormal (kept <= 128)
    // normal: kept in [128, 256]; a carry to 256 moves into the exponent
    uint32_t bits = ((uint32_t)(e + 127) << 7) + (uint32_t)(kept - 128);
    if (bits >= 0x7f80u) return sign | 0x7f80u;                    // overflow
    return sign | (uint16_t)bits;
}

__device__ inline float bf16_to_f32(uint16_t b) {
    return __uint_as_float((uint32_t)b << 16);
}

// Semirings of the product (MXE_SR_* in mxe.h: 0 (+, *), 1 (min, +), 2 (or,
// and)), Section 2: identity of the sum, the product of a value and an x, the
// sum. min and or are exact; a min accumulator only ever takes a smaller
// term, so it never turns NaN.
template <int SR, typename T> struct Semiring;
template <typename T> struct Semiring<0, T> {
    __device__ static T identity() { return T(0); }
    __device__ static T mul(T a, T x) { return a * x; }
    __device__ static T add(T p, T q) { return p + q; }
};
template <typename T> struct Semiring<1, T> {
    __device__ static T identity() { return T(__builtin_inf()); }
    __device__ static T mul(T a, T x) { return a + x; }
    __device__ static T add(T p, T q) { return q < p ? q : p; }
};
template <typename T> struct Semiring<2, T> {
    __device__ static T identity() { return T(0); }
    __device__ static T mul(T a, T x) { return (a != T(0) && x != T(0)) ? T(1) : T(0); }
    __device__ static T add(T p, T q) { return (p != T(0) || q != T(0)) ? T(1) : T(0); }
};

// Inclusive segmented scan over a wavefront whose keys never decrease
// (equal keys are adjacent; real keys stay below 0xfffffffe, padding lanes
// carry 0xffffffff after every real one), on DPP lane moves instead of LDS
// permutes:
// four row_shr steps inside each row of 16 lanes, then row_bcast:15 into rows
// 1 and 3 and row_bcast:31 into rows 2 and 3. A lane adds the moved value only
// when it carries its own key; moves from outside a row read key 0 and value
// 0 (adding nothing), and rows a broadcast skips keep a key no row can have.
// CTRL: a row shift, row_shr:n (0x110 + n) or row_shl:n (0x100 + n)
template <int CTRL>
__device__ inline uint32_t dpp_shr_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}
template <int CTRL, int RMASK>
__device__ inline uint32_t dpp_bcast_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0xfffffffeu, (int)v, CTRL, RMASK, 0xf, false);
}
template <int CTRL>
__device__ inline double dpp_shr(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp_shr(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL, int RMASK>
__device__ inline double dpp_bcast(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int RMASK>
__device__ inline float dpp_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RMASK, 0xf, false));
}

template <int CTRL, typename T, int KM>
__device__ inline void scan_shr(uint32_t key, T (&v)[KM]) {
    if constexpr (sizeof(T) == 4) {
        // FP32: each lane zeroes what the lane n places on in its row must
        // not take (the row_shl:n move of the key gives that lane's key), so
        // the move folds into a DPP add: two instructions per value, not
        // three. The same terms are added in the same order.
        constexpr int kShl = CTRL - 0x10;                     // row_shl:n for row_shr:n
        const bool keep = dpp_shr_u32<kShl>(key) == key;
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            const T w = keep ? v[q] : T(0);
            v[q] += dpp_shr<CTRL>(w);
        }
    } else {
        const bool take = dpp_shr_u32<CTRL>(key) == key;
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            const T m = dpp_shr<CTRL>(v[q]);
            v[q] += take ? m : T(0);
        }
    }
}
template <int CTRL, int RMASK, typename T, int KM>
__device__ inline void scan_bcast(uint32_t key, T (&v)[KM]) {
    const bool take = dpp_bcast_u32<CTRL, RMASK>(key) == key;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
        const T m = dpp_bcast<CTRL, RMASK>(v[q]);
        v[q] += take ? m : T(0);
    }
}
// The same scan for an operator other than +: every move, inside a row too,
// reads the operator's identity and the never-matching key where its source
// lane lies outside the row (for min, a moved-in 0 would be wrong).
template <int CTRL, int RMASK, typename Op, typename T, int KM>
__device__ inline void scan_step_op(uint32_t key, T (&v)[KM]) {
    const bool take = (uint32_t)__builtin_amdgcn_update_dpp((int)0xfffffffeu, (int)key, CTRL, RMASK,
                                                            0xf, false) == key;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
        T m;
        if constexpr (sizeof(T) == 8) {
            const double id = Op::identity();
            const int lo = __builtin_amdgcn_update_dpp(__double2loint(id), __double2loint(v[q]), CTRL,
                                                       RMASK, 0xf, false);
            const int hi = __builtin_amdgcn_update_dpp(__double2hiint(id), __double2hiint(v[q]), CTRL,
                                                       RMASK, 0xf, false);
            m = __hiloint2double(hi, lo);
        } else {
            m = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int((float)Op::identity()),
                                                           __float_as_int(v[q]), CTRL, RMASK, 0xf,
                                                           false));
        }
        v[q] = take ? Op::add(v[q], m) : v[q];
    }
}
template <typename Op, typename T, int KM>
__device__ inline void segmented_scan_op(uint32_t key, T (&v)[KM]) {
    scan_step_op<0x111, 0xf, Op>(key, v);
    scan_step_op<0x112, 0xf, Op>(key, v);
    scan_step_op<0x114, 0xf, Op>(key, v);
    scan_step_op<0x118, 0xf, Op>(key, v);
    scan_step_op<0x142, 0xa, Op>(key, v);
    scan_step_op<0x143, 0xc, Op>(key, v);
}

template <typename T, int KM>
__device__ inline void segmented_scan(uint32_t key, T (&v)[KM]) {
    scan_shr<0x111>(key, v);            // row_shr:1
    scan_shr<0x112>(key, v);            // row_shr:2
    scan_shr<0x114>(key, v);            // row_shr:4
    scan_shr<0x118>(key, v);            // row_shr:8
    scan_bcast<0x142, 0xa>(key, v);     // row_bcast:15 -> rows 1, 3
    scan_bcast<0x143, 0xc>(key, v);     // row_bcast:31 -> rows 2, 3
}

}  // namespace mxe
