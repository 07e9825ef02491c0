/*
 * mxe — max-entropy permuted sparse matrix-vector product on MI355X (gfx950).
 *
 * C ABI of libmxe.so. The library implements the method of Jain et al.,
 * "Entropy Maximization in Sparse Matrix by Vector Multiplication": permute
 * the rows and columns of a CSR matrix at random, (P_r y) = (P_r A P_c)(P_c^-1 x)
 * (Section 1, Eq. 1; Section 3), measure how evenly the nonzeros spread with
 * the Shannon entropy of a 2D block histogram (Section 4, Eq. eq:entropy;
 * Section 5), and multiply the permuted, resident matrix by dense vectors
 * (Section 2). Every step runs in HIP kernels on the GPU.
 *
 * Conventions shared by every call
 *   - Matrices are canonical CSR (Section 2): row_ptr[nrows+1] int32 with
 *     row_ptr[0] = 0, nondecreasing, row_ptr[nrows] = nnz; col_idx[nnz] int32 in
 *     [0, ncols), strictly increasing inside a row (duplicates are rejected);
 *     explicit zeros are kept and count as entries. nnz < 2^31.
 *   - Permutations are in new-to-old (gather) form: row i' of B = P_r A P_c is
 *     row rperm[i'] of A, column j' of B is column cperm[j'] of A. Hence
 *     x' = P_c^-1 x is x'[j'] = x[cperm[j']] and y' = P_r y is y'[i'] = y[rperm[i']].
 *   - Dense operands X (ncols x k) and Y (nrows x k) are row-major with leading
 *     dimension ld >= k, in device memory owned by the caller. They are FP64
 *     for matrices stored in MXE_F64 and FP32 for MXE_F32 / MXE_BF16 storage.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *     taking a stream are stream-ordered and return before the device work ends,
 *     unless stated otherwise.
 *   - Errors are reported by status only; nothing throws across the ABI. A
 *     failing call leaves its outputs unspecified and changes no handle.
 *     mxe_last_error() returns this thread's detail text for the last failure.
 *   - Calls on one context are serialized internally; mxe_submit and mxe_wait
 *     may be called from any thread.
 */
#ifndef MXE_H
#define MXE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MXE_ABI_VERSION 1

typedef enum mxe_status {
    MXE_OK = 0,
    MXE_ERR_INVALID_ARG = 1,    /* a NULL pointer, negative size, k < 1, ld < k, grid out of range */
    MXE_ERR_INVALID_CSR = 2,    /* row_ptr / col_idx break the canonical CSR rules above */
    MXE_ERR_NOT_FOUND = 3,      /* unknown or released handle */
    MXE_ERR_BUSY = 4,           /* release of a matrix with queued or running work */
    MXE_ERR_BUDGET = 5,         /* the HBM budget given to mxe_create would be exceeded */
    MXE_ERR_OUT_OF_MEMORY = 6,  /* device allocation failed */
    MXE_ERR_UNSUPPORTED = 7,    /* valid request this build does not handle */
    MXE_ERR_TIMEOUT = 8,        /* mxe_wait timed out; the request is still live */
    MXE_ERR_DEVICE = 9,         /* HIP runtime error or no usable gfx950 device */
    MXE_ERR_INEXACT = 10        /* entropy: correct rounding could not be certified */
} mxe_status;

typedef enum mxe_dtype {        /* storage type of matrix values */
    MXE_F64 = 0,
    MXE_F32 = 1,                /* rounded once, to nearest-even, from the FP64 input */
    MXE_BF16 = 2                /* rounded once, to nearest-even, from the FP64 input */
} mxe_dtype;

/* flags */
#define MXE_INPUT_DEVICE    0x1u  /* register: the three arrays are device pointers */
#define MXE_OUTPUT_DEVICE   0x1u  /* get_permutation / export: outputs are device pointers */
#define MXE_ROWS            0x1u  /* permute mode: random row permutation ("R") */
#define MXE_COLS            0x2u  /* permute mode: random column permutation */
#define MXE_GRADIENT        0x4u  /* permute mode: gradient-based shuffles (G-R, G-C) */
#define MXE_SPACE_PERMUTED  0x0u  /* spmv: X, Y are in the permuted index space */
#define MXE_SPACE_ORIGINAL  0x1u  /* spmv: X, Y are in A's index space (gather/scatter inside) */

typedef struct mxe_ctx mxe_ctx;
typedef int64_t mxe_mat;        /* matrix handle, > 0 */
typedef int64_t mxe_plan;       /* batch plan handle, > 0 */
typedef int64_t mxe_ticket;     /* serving request handle, > 0 */

typedef struct mxe_matrix_desc {
    int32_t nrows, ncols;
    int64_t nnz;
    int32_t storage;            /* mxe_dtype */
    int32_t permuted;           /* 1 if made by mxe_permute */
    mxe_mat parent;             /* the matrix it was permuted from, else 0 */
    uint64_t seed;              /* permute seed, else 0 */
    uint32_t mode;              /* permute mode, else 0 */
    uint64_t device_bytes;      /* HBM held for this matrix */
    int32_t max_row;            /* longest row */
    double mean_row;            /* nnz / nrows */
} mxe_matrix_desc;

/* --- library and context -------------------------------------------------- */

const char *mxe_status_string(mxe_status s);
/* Detail of this thread's last failed call; never NULL; valid until the next call. */
const char *mxe_last_error(void);
int32_t mxe_abi_version(void);

/* Creates a context on HIP device `device`. hbm_budget_bytes caps the HBM the
 * context holds for resident matrices and in-flight serving work (0 = no cap).
 * Returns MXE_ERR_DEVICE if the device is missing or is not gfx950. */
mxe_status mxe_create(int32_t device, uint64_t hbm_budget_bytes, mxe_ctx **out);
/* Waits for all work, stops the serving loop, frees every matrix and plan. */
mxe_status mxe_destroy(mxe_ctx *ctx);

/* Checks canonical CSR (Section 2) on the host; needs no device or context.
 * Returns MXE_OK, MXE_ERR_INVALID_ARG or MXE_ERR_INVALID_CSR. */
mxe_status mxe_validate_csr(int32_t nrows, int32_t ncols, int64_t nnz,
                            const int32_t *row_ptr, const int32_t *col_idx);

/* --- matrices --------------------------------------------------------------- */

/* Copies a CSR matrix into HBM, storing values as `storage`. Host inputs are
 * validated before any device work; device inputs (MXE_INPUT_DEVICE) are
 * validated after a staging copy of row_ptr and col_idx. The caller may free
 * its arrays when the call returns (it synchronizes). Values are FP64. */
mxe_status mxe_register_matrix(mxe_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz,
                               const int32_t *row_ptr, const int32_t *col_idx,
                               const double *vals, mxe_dtype storage, uint32_t flags,
                               mxe_mat *out);

/* The randomization of Section 3 / Eq. 1: B = P_r A P_c in canonical CSR,
 * with P_r drawn when mode has MXE_ROWS and P_c when it has MXE_COLS (identity
 * otherwise). The permutation of n items is the stable ascending order of n
 * 64-bit keys, key(i) = i-th output of SplitMix64 started at the stream seed;
 * the row stream's seed is the first SplitMix64 output started at `seed`, the
 * column stream's the second. Equal seeds give bit-identical B. B's rows are
 * re-sorted by new column; values move bit-exactly. B holds A alive.
 * With MXE_GRADIENT the rows (MXE_ROWS) and/or columns (MXE_COLS) take
 * Section 8's gradient formats instead (G-R, G-C): with h the nonzeros per
 * row (per column), the pivot p is the first index of the maximum of
 * h[i+1] - h[i]; the parts [0, p] and [p+1, n) are each ordered by the
 * stream's keys (random order within each part) and riffled, the two parts
 * alternating and the longer part's remainder appended. Synchronizes
 * `stream` once per gradient shuffle (the pivot sizes the parts). */
mxe_status mxe_permute(mxe_ctx *ctx, mxe_mat a, uint64_t seed, uint32_t mode,
                       void *stream, mxe_mat *out_b);

/* Copies B's permutations (new-to-old, nrows / ncols int32) to host memory,
 * or device memory with MXE_OUTPUT_DEVICE; either pointer may be NULL.
 * Synchronizes `stream`. For an unpermuted matrix both are the identity. */
mxe_status mxe_get_permutation(mxe_ctx *ctx, mxe_mat b, int32_t *rperm, int32_t *cperm,
                               uint32_t flags, void *stream);

/* Copies the stored CSR out (vals in the storage type: double, float or
 * uint16 BF16 bits). Host outputs unless MXE_OUTPUT_DEVICE. Synchronizes. */
mxe_status mxe_export_csr(mxe_ctx *ctx, mxe_mat m, int32_t *row_ptr, int32_t *col_idx,
                          void *vals, uint32_t flags, void *stream);

mxe_status mxe_matrix_info(mxe_ctx *ctx, mxe_mat m, mxe_matrix_desc *out);

/* Releases a handle. A permuted matrix keeps its parent's memory until it is
 * released too, and a batch plan keeps its matrices' memory until the plan is
 * destroyed. Returns MXE_ERR_BUSY while serving work on it is queued or
 * running. When the last reference to a matrix's memory goes, the call waits
 * for the work that library calls queued on that matrix (on each stream they
 * used, up to its last such call) before the memory is freed; it does not
 * wait for the rest of the device. */
mxe_status mxe_release(mxe_ctx *ctx, mxe_mat m);

/* --- measure (Sections 4 and 5) --------------------------------------------- */

/* Block-grid nonzero entropy. Entry (i, j) falls in block
 * (floor(i*grid_rows/nrows), floor(j*grid_cols/ncols)), computed exactly;
 * H = -sum p log p over bins with p = count / nnz > 0 (Eq. eq:entropy),
 * returned correctly rounded to FP64 in bits (h_bits) and nats (h_nats,
 * may be NULL). An empty matrix, or one whose entries share one block, has
 * H = 0. hist (grid_rows*grid_cols int64, row-major, host memory) may be NULL.
 * 1 <= grid_rows, grid_cols <= 2^20. Synchronizes `stream`. Returns
 * MXE_ERR_INEXACT (values still written) in the rare case that the
 * double-double evaluation cannot certify the rounding. */
mxe_status mxe_entropy(mxe_ctx *ctx, mxe_mat m, int32_t grid_rows, int32_t grid_cols,
                       void *stream, double *h_bits, double *h_nats, int64_t *hist);

/* Hierarchical 2D entropy (Section 5: 2x2, 4x4 and 8x8 heat maps, fewer
 * regions where the grid is smaller). For each of the nlevels levels L the
 * grid_rows x grid_cols block histogram is cut into Lr x Lc regions,
 * Lr = min(L, grid_rows), Lc = min(L, grid_cols); region (a, b) holds the
 * bins (r, c) with floor(r*Lr/grid_rows) = a and floor(c*Lc/grid_cols) = b,
 * and its entropy is that of its own bins, correctly rounded as in
 * mxe_entropy. h_bits / h_nats (host, nats may be NULL) receive the levels
 * one after another, each Lr x Lc row-major. 1 <= L <= 64. Synchronizes.
 * Returns MXE_ERR_INEXACT (values written) if any rounding is uncertified. */
mxe_status mxe_entropy_levels(mxe_ctx *ctx, mxe_mat m, int32_t grid_rows, int32_t grid_cols,
                              const int32_t *levels, int32_t nlevels, void *stream,
                              double *h_bits, double *h_nats);

/* --- products (Section 2) --------------------------------------------------- */

/* Y = M X for one matrix, k >= 1 right-hand sides (X: ncols x k, Y: nrows x k).
 * For a permuted B and MXE_SPACE_ORIGINAL, X and Y are in A's index space:
 * the call gathers X by cperm, multiplies, and scatters Y by rperm (Eq. 1).
 * FP64 storage accumulates in FP64; FP32/BF16 storage accumulates in FP32.
 * The kernel variant is the autotuned one for (matrix, k) (mxe_tune). */
mxe_status mxe_spmv(mxe_ctx *ctx, mxe_mat m, int32_t k, const void *X, int64_t ldx,
                    void *Y, int64_t ldy, uint32_t flags, void *stream);

/* Semirings for mxe_spmv_semiring (Section 2 defines the product on (+, *)
 * and notes it extends to others). */
#define MXE_SR_PLUS_TIMES 0   /* y_i = sum of v * x: the same as mxe_spmv */
#define MXE_SR_MIN_PLUS   1   /* y_i = min over row i's stored entries of v + x; +inf if none */
#define MXE_SR_OR_AND     2   /* y_i = 1 if a stored v != 0 meets x != 0 in row i, else 0 */

/* Y = M X over `semiring`, otherwise as mxe_spmv (k >= 1, index spaces,
 * storage and accumulation types); the kernel is the column-slab one when the
 * matrix's autotuned (+, *) variant for k is (tuning first if needed), else
 * a row-group kernel. (min, +) and (or, and) results do not depend on the
 * order of the terms, so they are exact: the same bits as a sequential loop
 * over each row in the accumulation type. */
mxe_status mxe_spmv_semiring(mxe_ctx *ctx, mxe_mat m, int32_t semiring, int32_t k, const void *X,
                             int64_t ldx, void *Y, int64_t ldy, uint32_t flags, void *stream);

/* x' = P_c^-1 x: Xp[j'] = X[cperm[j']] (k columns). */
mxe_status mxe_gather_x(mxe_ctx *ctx, mxe_mat b, int32_t k, const void *X, int64_t ldx,
                        void *Xp, int64_t ldxp, void *stream);
/* y = P_r^-1 y': Y[rperm[i']] = Yp[i'] (k columns). */
mxe_status mxe_scatter_y(mxe_ctx *ctx, mxe_mat b, int32_t k, const void *Yp, int64_t ldyp,
                         void *Y, int64_t ldy, void *stream);

/* SpMV kernel variants. A variant id packs the kernel family and its lane
 * count per row: family MXE_VAR_GROUP with lanes 1..64 (rows per wavefront =
 * 64 / lanes), MXE_VAR_BINNED (row-length bins, each with its own lanes), or
 * MXE_VAR_MERGE (merge-path split of rows + nonzeros, equal work per group), or
 * MXE_VAR_SLAB with lanes = slab size in units of 64 KiB (1..64): a column-slab layout,
 * built once per matrix and right-hand-side class, whose workgroups keep
 * their rows' partial sums in LDS and gather x one L2-sized slab at a time;
 * row blocks are sized for two workgroups per compute unit, or for one when
 * MXE_SLAB_ONE_PER_CU is added to the slab size. */
#define MXE_VAR_GROUP   0x000
#define MXE_VAR_BINNED  0x100
#define MXE_VAR_MERGE   0x200
#define MXE_VAR_SLAB    0x300
#define MXE_SLAB_ONE_PER_CU 0x80
/* MXE_VAR_FIXED with lanes per row (1..64): Section 7's equal-row split, a
 * fixed grid of 2048 workgroups each owning an equal contiguous share of rows,
 * nothing rebalanced (the case where the paper sees randomization help). */
#define MXE_VAR_FIXED   0x400
/* MXE_VAR_COO (lanes ignored, 0): Section 2's coordinate format. The first
 * use builds a row index per stored entry (4 bytes per nonzero, counted in
 * the HBM budget, kept until the matrix is released); every 256-entry tile
 * is reduced by row and the rows cut by a tile edge are joined by a second
 * pass. Never chosen by mxe_tune; force it with mxe_set_variant. */
#define MXE_VAR_COO     0x500
/* MXE_VAR_WINDOW with the lanes of MXE_VAR_SLAB (slab size, one-per-CU
 * flag): the same column-slab layout, plus a window of x held in LDS for each
 * row block: the widest range of columns that fits the workgroup's LDS beside
 * its partial sums, placed (once, when first used) where a sample of the
 * block's stored columns is densest. Entries inside the window read x from
 * LDS, the others gather it as MXE_VAR_SLAB does. It pays off when a row
 * block's columns cluster (the unpermuted, mostly diagonal matrices of
 * Section 7), not after the max-entropy permutation spreads them. */
#define MXE_VAR_WINDOW  0x600
#define MXE_VARIANT(family, lanes) ((family) | (lanes))

/* Measures the device's random 8-byte gather rate, the ceiling of a sparse
 * product whose x reads are scattered (Section 3's max-entropy matrices): a
 * kernel issues about `gathers` loads at LCG-drawn positions of a zeroed
 * table of `table_bytes` (8 .. 2^34, a multiple of 64), each XCD confined to
 * its own eighth of the table when per_xcd != 0 (as the column-slab product
 * confines it to a slab). *gathers_per_s = loads issued / kernel time (HIP
 * events on `stream`). Allocates the table from the stream-ordered pool;
 * synchronizes. A diagnostic: no result of the method depends on it. */
mxe_status mxe_probe_gather(mxe_ctx *ctx, int64_t table_bytes, int64_t gathers, int32_t per_xcd,
                            void *stream, double *gathers_per_s);

/* Times the candidate variants for (m, k) on the device (each briefly, then
 * the closest few again, interleaved) and caches the fastest; returns it in
 * *variant (may be NULL). Synchronizes. */
mxe_status mxe_tune(mxe_ctx *ctx, mxe_mat m, int32_t k, void *stream, int32_t *variant);
/* Forces a variant for (m, k); variant 0 clears the choice (retune on use).
 * MXE_ERR_INVALID_ARG for an unknown family, lanes out of range, or bits
 * above the family; MXE_ERR_UNSUPPORTED when the variant cannot run on this
 * matrix (a slab layout that does not fit, merge-path with k > 4). */
mxe_status mxe_set_variant(mxe_ctx *ctx, mxe_mat m, int32_t k, int32_t variant);

/* --- batches: many matrices, one persistent launch ------------------------- */

typedef struct mxe_item {
    mxe_mat mat;
    int32_t k;
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    uint32_t flags;             /* MXE_SPACE_PERMUTED only in batches */
} mxe_item;

/* The reuse setting of Section 1: randomization is a cheap preconditioning
 * of the product, paid once and repaid over the many products an iterative
 * solver (or a convolution) takes with the same resident matrix; Section 7
 * ("randomization sometimes works") makes the same point. A batch runs many
 * such products at once: Y_i = M_i X_i for every item (Section 2's product,
 * k_i <= 16 right-hand sides each, permuted index space only, each X_i / Y_i
 * laid out as for mxe_spmv). One persistent launch computes every item: the
 * items are cut into work units (slab-layout blocks or row tiles), dealt to
 * one work queue per XCD, and workgroups pull units from their own XCD's
 * queue, then from the others. Stream-ordered on `stream`; the call builds
 * its work list on the host and may tune items first (as mxe_tune).
 * MXE_ERR_UNSUPPORTED for k > 16 or MXE_SPACE_ORIGINAL items; every item is
 * validated before any launch. */
mxe_status mxe_spmv_batch(mxe_ctx *ctx, int32_t count, const mxe_item *items, void *stream);

/* Section 1's reuse, repeated: the same batch of products on resident
 * matrices, again and again. mxe_batch_create plans a batch once (autotunes
 * each item, builds the work list) and captures the launch in a HIP graph
 * (synchronizes); mxe_batch_launch replays it on `stream` (stream-ordered).
 * Items passed to launch must name the same matrices and k in the same
 * order; their X / Y pointers may change (the descriptor table is rewritten
 * on the device, ordered after the previous replay). items == NULL replays
 * with the current pointers. Replays of one plan never overlap: each waits
 * on the device for the previous one, whatever stream that ran on. The plan
 * keeps its matrices alive until mxe_batch_destroy, which waits for the last
 * replay. */
mxe_status mxe_batch_create(mxe_ctx *ctx, int32_t count, const mxe_item *items, mxe_plan *out);
mxe_status mxe_batch_launch(mxe_ctx *ctx, mxe_plan plan, const mxe_item *items, void *stream);
mxe_status mxe_batch_destroy(mxe_ctx *ctx, mxe_plan plan);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Computes
 * what mxe_spmv_batch computes, with the same kernel, work units and queues
 * (so the same bits), but allocates no device memory: the descriptor table,
 * queue entries and queue counters live in a static device array of
 * MXE_NOALLOC_SCRATCH_BYTES that the library keeps on every GPU it runs on
 * until the process ends, which limits a call to MXE_NOALLOC_MAX_ITEMS items.
 * Nothing is tuned or built here: every item's matrix must already be tuned
 * for its k (MXE_ERR_UNSUPPORTED naming the item otherwise), and an item runs
 * on the layout that an earlier mxe_spmv_batch or mxe_batch_create with the
 * same matrix and k built; call one of them once with the same items first to
 * get its result bit for bit. count above MXE_NOALLOC_MAX_ITEMS:
 * MXE_ERR_INVALID_ARG. Stream-ordered on `stream`; the descriptor table is
 * copied from host memory on that stream, and the call returns once the copy
 * has taken its data. Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (the counters are cleared by a kernel on
 * `stream` before each use): calls whose work may overlap on one GPU (other
 * streams, threads or contexts) race on it and must be ordered by the
 * caller; calls on one stream are ordered already. */
#define MXE_NOALLOC_MAX_ITEMS 256
#define MXE_NOALLOC_SCRATCH_BYTES 65536
mxe_status mxe_spmv_batch_noalloc(mxe_ctx *ctx, int32_t count, const mxe_item *items,
                                  void *stream);

/* --- serving: continuous batching of requests on resident matrices -------- */

#define MXE_SERVE_MAX_BATCH 64

typedef struct mxe_serve_config {
    int32_t streams;            /* device streams the loop issues on (>= 1) */
    int32_t max_inflight;       /* items (products) on the device at once (>= 1) */
    int32_t max_batch;          /* items per launch (1..MXE_SERVE_MAX_BATCH) */
    int32_t max_merge_k;        /* right-hand sides of a merged item (1..16; 1: no merging) */
} mxe_serve_config;

/* Starts the serving loop (one scheduler thread and `streams` device
 * streams, each with a device descriptor table, its pinned twin and, when
 * max_merge_k > 1, a staging matrix for merged right-hand sides: twice the
 * widest resident matrix's columns times max_merge_k rounded up to a power of
 * two, at least 64 MiB, counted in the HBM budget; all allocated here). Requests are admitted
 * in arrival order while the in-flight vector bytes fit the context budget
 * beside the resident matrices. Each admission round takes up to max_batch
 * items, each taking one of max_inflight slots: an item is one request, or
 * queued permuted-space requests on the same matrix merged into one product
 * of at most max_merge_k right-hand sides (the matrix streams once for all of
 * them; their X are packed into the staging by one kernel per round and each
 * result column is written into its own request's Y); a request merged into
 * an item takes no slot of its own. A round of one
 * unmerged request runs as its own autotuned product (as mxe_spmv);
 * otherwise the permuted-space items run as one persistent launch of
 * mxe_spmv_batch's kernel on the least-loaded stream whose table is free,
 * and original-space or k > 16 requests as their own products. With
 * max_batch 1 and max_merge_k 1 every request runs exactly as mxe_spmv would
 * run it. Launches on different streams overlap on the device. The
 * scheduler thread polls without sleeping while products run and for 2 ms
 * after the last one ends (a woken thread would add tens of microseconds to
 * a lone request), then sleeps until the next submission: it keeps one host
 * core busy under load.
 * MXE_ERR_BUDGET when the staging does not fit the budget. */
mxe_status mxe_serve_start(mxe_ctx *ctx, const mxe_serve_config *cfg);
/* Serving is Section 1's reuse as a service: matrices are permuted once and
 * stay resident; each request is one product Y = M X (Section 2; Eq. 1 when
 * flags is MXE_SPACE_ORIGINAL), k >= 1 right-hand sides laid out as for
 * mxe_spmv. Queues a request and returns its ticket at once (X, Y stay owned
 * by the caller and must stay alive until mxe_wait returns for it; the
 * matrix's own creation, e.g. the stream given to mxe_permute, must be
 * complete). The first request on a matrix for a k class tunes the matrix
 * for it (and for each larger class a merge can reach) and builds the layouts
 * a batch runs it on, here in the submitting thread, so the scheduler only
 * looks them up. MXE_ERR_INVALID_ARG for a bad
 * request or no running loop, MXE_ERR_NOT_FOUND for an unknown matrix.
 * Thread-safe. */
mxe_status mxe_submit(mxe_ctx *ctx, const mxe_item *req, mxe_ticket *out);
/* The completion side of a Section 1 reuse request (see mxe_submit). Blocks
 * until the request is done (timeout_us < 0: forever). On return other than
 * MXE_ERR_TIMEOUT the ticket is retired; on MXE_OK *latency_us (may be NULL)
 * holds submit-to-completion time, else the status is the request's own
 * failure (MXE_ERR_BUDGET for a request that can never fit the budget).
 * MXE_ERR_TIMEOUT leaves the ticket live. Thread-safe. */
mxe_status mxe_wait(mxe_ctx *ctx, mxe_ticket t, int64_t timeout_us, double *latency_us);
/* Drains queued and running requests, then stops the loop. */
mxe_status mxe_serve_stop(mxe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MXE_H */
