/*
 * CPU oracle for max-entropy permuted SpMV — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct implementation of what the GPU path
 * computes, written from the paper (Jain et al., "Entropy Maximization in
 * Sparse Matrix by Vector Multiplication"). Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it. It shares no code, header
 * or constant table with the GPU library.
 *
 * Every function states the passage it follows. Where the paper is silent the
 * reading taken is stated next to the code.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC mxe_oracle.c -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random keys.                                                             */
/*                                                                          */
/* Section 3 defines randomization as a row or column permutation chosen by */
/* a pseudo-random process; the paper draws it with a time-seeded numpy     */
/* generator, which cannot be reproduced. Reading taken: the random         */
/* permutation is the stable argsort of one 64-bit pseudo-random key per    */
/* index, the keys being consecutive outputs of SplitMix64 (Steele, Lea and */
/* Flood, OOPSLA 2014), implemented here from its published definition:     */
/* the state advances by the golden-ratio increment before each output, and */
/* each output is the state passed through the variant-13 finaliser.        */
/* ------------------------------------------------------------------------ */

/* Writes the first n outputs of the SplitMix64 generator started at state s. */
void orc_splitmix64_outputs(uint64_t s, int64_t n, uint64_t *out)
{
    uint64_t state = s;
    for (int64_t i = 0; i < n; ++i) {
        state += 0x9e3779b97f4a7c15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        out[i] = z ^ (z >> 31);
    }
}

/* The row stream's seed is the first output of SplitMix64 started at the
 * user seed, the column stream's seed the second. */
void orc_stream_seeds(uint64_t seed, uint64_t *s_row, uint64_t *s_col)
{
    uint64_t two[2];
    orc_splitmix64_outputs(seed, 2, two);
    *s_row = two[0];
    *s_col = two[1];
}

/* ------------------------------------------------------------------------ */
/* Permutation = stable argsort of the keys (Section 3, Eq. 1).             */
/* perm is in new-to-old (gather) form: position k of the permuted order    */
/* holds original index perm[k]. Equal keys keep index order.               */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t idx; } orc_keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const orc_keyidx *x = (const orc_keyidx *)a, *y = (const orc_keyidx *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/* Returns 0 on success, -1 if memory runs out. */
int orc_argsort_keys(int64_t n, const uint64_t *keys, int32_t *perm)
{
    orc_keyidx *t = (orc_keyidx *)malloc((size_t)(n > 0 ? n : 1) * sizeof *t);
    if (!t) return -1;
    for (int64_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].idx = i; }
    qsort(t, (size_t)n, sizeof *t, cmp_keyidx);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)t[i].idx;
    free(t);
    return 0;
}

/* inv[perm[k]] = k: the old-to-new form of the same permutation. */
void orc_invert(int64_t n, const int32_t *perm, int32_t *inv)
{
    for (int64_t k = 0; k < n; ++k) inv[perm[k]] = (int32_t)k;
}

/* ------------------------------------------------------------------------ */
/* Permuted matrix B = P_r A P_c (Eq. 1) in canonical CSR (Section 2).      */
/* Row k of B is row rperm[k] of A; an entry in column j of A moves to      */
/* column cinv[j]. The paper keeps CSR columns increasing within a row      */
/* (Section 2) but is silent on re-sorting after the column permutation;    */
/* reading taken: B is canonical, so each row is re-sorted by new column.   */
/* Values move unchanged.                                                   */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t col; double val; } orc_colval;

static int cmp_colval(const void *a, const void *b)
{
    const orc_colval *x = (const orc_colval *)a, *y = (const orc_colval *)b;
    return (x->col > y->col) - (x->col < y->col);
}

int orc_permute_csr(int32_t nrows, const int32_t *rp, const int32_t *col,
                    const double *val, const int32_t *rperm, const int32_t *cinv,
                    int32_t *rp_out, int32_t *col_out, double *val_out)
{
    int64_t maxlen = 0;
    for (int32_t i = 0; i < nrows; ++i)
        if (rp[i + 1] - rp[i] > maxlen) maxlen = rp[i + 1] - rp[i];
    orc_colval *row = (orc_colval *)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof *row);
    if (!row) return -1;
    int64_t pos = 0;
    rp_out[0] = 0;
    for (int32_t k = 0; k < nrows; ++k) {
        int32_t src = rperm[k];
        int64_t len = rp[src + 1] - rp[src];
        for (int64_t t = 0; t < len; ++t) {
            row[t].col = cinv[col[rp[src] + t]];
            row[t].val = val[rp[src] + t];
        }
        qsort(row, (size_t)len, sizeof *row, cmp_colval);
        for (int64_t t = 0; t < len; ++t) {
            col_out[pos + t] = row[t].col;
            val_out[pos + t] = row[t].val;
        }
        pos += len;
        rp_out[k + 1] = (int32_t)pos;
    }
    free(row);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2D block histogram (Section 4, the heat-map histogram; Section 5, the    */
/* hierarchical 2D view). The paper fixes neither the bin count nor the     */
/* mapping. Reading taken: a G_r x G_c grid with proportional mapping,      */
/* block-row floor(i G_r / M) and block-column floor(j G_c / N), in exact   */
/* integer arithmetic. Each stored entry counts once.                       */
/* ------------------------------------------------------------------------ */

void orc_block_hist(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *col,
                    int32_t grid_r, int32_t grid_c, int64_t *hist)
{
    memset(hist, 0, (size_t)grid_r * (size_t)grid_c * sizeof *hist);
    for (int32_t i = 0; i < nrows; ++i) {
        int64_t bi = (int64_t)i * grid_r / nrows;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t bj = (int64_t)col[e] * grid_c / ncols;
            hist[bi * grid_c + bj] += 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* SpMV and SpMM over (+, *) in FP64 (Section 2): y_i is the sum over the   */
/* stored entries of row i of V[l] * x[COL[l]], added left to right in      */
/* storage order. (The printed sum has x's index typo'd as y's.)            */
/* X is row-major nrows_x by k with leading dimension ldx; so is Y.         */
/* ------------------------------------------------------------------------ */

void orc_spmm(int32_t nrows, const int32_t *rp, const int32_t *col, const double *val,
              int32_t k, const double *x, int64_t ldx, double *y, int64_t ldy)
{
    for (int32_t i = 0; i < nrows; ++i) {
        for (int32_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                acc += val[e] * x[(int64_t)col[e] * ldx + c];
            y[(int64_t)i * ldy + c] = acc;
        }
    }
}

/* SpMV / SpMM over other semirings (Section 2 notes the product extends to */
/* them): (min, +), y_i = min over row i's stored entries of V[l] + x[COL[l]] */
/* (+inf for an empty row, the shortest-path step), and Boolean (or, and),   */
/* y_i = 1 if some stored V[l] != 0 meets x[COL[l]] != 0, else 0             */
/* (reachability). min and or are exact, so the order does not matter.      */
void orc_spmm_min_plus(int32_t nrows, const int32_t *rp, const int32_t *col, const double *val,
                       int32_t k, const double *x, int64_t ldx, double *y, int64_t ldy)
{
    for (int32_t i = 0; i < nrows; ++i) {
        for (int32_t c = 0; c < k; ++c) {
            double acc = INFINITY;
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                double t = val[e] + x[(int64_t)col[e] * ldx + c];
                if (t < acc) acc = t;
            }
            y[(int64_t)i * ldy + c] = acc;
        }
    }
}

void orc_spmm_or_and(int32_t nrows, const int32_t *rp, const int32_t *col, const double *val,
                     int32_t k, const double *x, int64_t ldx, double *y, int64_t ldy)
{
    for (int32_t i = 0; i < nrows; ++i) {
        for (int32_t c = 0; c < k; ++c) {
            int any = 0;
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                if (val[e] != 0.0 && x[(int64_t)col[e] * ldx + c] != 0.0) any = 1;
            y[(int64_t)i * ldy + c] = any ? 1.0 : 0.0;
        }
    }
}

/* COO SpMV / SpMM (Section 2's coordinate format): Y starts at zero and   */
/* every stored entry l, in storage order, adds V[l] * x[COL[l]] to row     */
/* ROW[l]. On entries sorted by row this adds each row's terms in the same  */
/* order as orc_spmm.                                                       */
void orc_coo_spmm(int32_t nrows, int64_t nnz, const int32_t *row, const int32_t *col,
                  const double *val, int32_t k, const double *x, int64_t ldx, double *y,
                  int64_t ldy)
{
    for (int32_t i = 0; i < nrows; ++i)
        for (int32_t c = 0; c < k; ++c)
            y[(int64_t)i * ldy + c] = 0.0;
    for (int64_t e = 0; e < nnz; ++e)
        for (int32_t c = 0; c < k; ++c)
            y[(int64_t)row[e] * ldy + c] += val[e] * x[(int64_t)col[e] * ldx + c];
}

/* Same arithmetic, rows split evenly over OpenMP threads with a static
 * schedule: the equal-row split of Section 7's parallel CSR experiment. It is
 * timed as the CPU baseline; its results equal orc_spmm's bit for bit. */
void orc_spmm_parallel(int32_t nrows, const int32_t *rp, const int32_t *col, const double *val,
                       int32_t k, const double *x, int64_t ldx, double *y, int64_t ldy)
{
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < nrows; ++i) {
        for (int32_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                acc += val[e] * x[(int64_t)col[e] * ldx + c];
            y[(int64_t)i * ldy + c] = acc;
        }
    }
}

int orc_omp_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Storage precision (beyond the paper, which is FP64 only): FP64 values    */
/* are rounded once, to nearest with ties to even, straight from FP64 to    */
/* the storage format. FP32 is the C conversion under the default rounding */
/* mode. BF16 (1 sign, 8 exponent, 7 fraction bits, the top half of an FP32 */
/* pattern) is rounded here from the FP64 value directly, never through     */
/* FP32, which would round twice.                                           */
/* ------------------------------------------------------------------------ */


void orc_round_f32(int64_t n, const double *in, float *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = (float)in[i];
}

static uint16_t f32_top_half(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return (uint16_t)(u >> 16);
}

uint16_t orc_bf16_from_f64(double d)
{
    if (isnan(d)) return (uint16_t)(signbit(d) ? 0xFFC0 : 0x7FC0);
    double a = fabs(d);
    uint16_t sign = signbit(d) ? 0x8000 : 0;
    if (isinf(a)) return sign | 0x7F80;
    /* spacing of BF16 values around a: 2^(e-7) for a in [2^e, 2^(e+1)),
     * e >= -126; below 2^-126 the subnormal spacing 2^-133 */
    double q;
    if (a < ldexp(1.0, -126)) {
        q = ldexp(1.0, -133);
    } else {
        int e;
        frexp(a, &e);            /* a = m 2^e, m in [0.5, 1) */
        q = ldexp(1.0, e - 1 - 7);
    }
    double lo = floor(a / q) * q;     /* largest multiple of q not above a */
    double hi = lo + q;
    double below = a - lo, above = hi - a;
    double r;
    if (below < above) r = lo;
    else if (above < below) r = hi;
    else r = (fmod(lo / q, 2.0) == 0.0) ? lo : hi;   /* tie: even multiple */
    /* largest finite BF16 is (2 - 2^-7) 2^127; anything rounding above it
     * becomes infinity */
    if (r > ldexp(2.0 - ldexp(1.0, -7), 127)) return sign | 0x7F80;
    return sign | f32_top_half((float)r);     /* r is exact in FP32 */
}

void orc_round_bf16(int64_t n, const double *in, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16_from_f64(in[i]);
}
