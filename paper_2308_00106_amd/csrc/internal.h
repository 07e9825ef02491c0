// Internal interfaces between the host runtime (api.cpp, serve.cpp) and the
// HIP kernels. Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mxe {

// ---- generic -------------------------------------------------------------
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_iota_i32(int32_t *p, int64_t n, hipStream_t s);

// Exclusive scan of n int32 values (in may equal out). The running total
// must stay below 2^31. Workspace: scan_ws_bytes(n).
size_t scan_ws_bytes(int64_t n);
hipError_t launch_exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *ws,
                                 hipStream_t s);

// ---- random permutation (keys + LDS radix / bucket sort) --------------------
// perm: new-to-old, inv: old-to-new. Workspace: random_perm_ws_bytes(n).
size_t random_perm_ws_bytes(int64_t n);
hipError_t launch_random_perm(int64_t n, uint64_t stream_seed, int32_t *perm, int32_t *inv,
                              void *ws, hipStream_t s);

// ---- gradient-based shuffle --------------------------------------------------
// counts[i] = nonzeros of row i (rows) or of column i (!rows, n = ncols).
hipError_t launch_line_counts(bool rows, int32_t nrows, int64_t nnz, const int32_t *rp,
                              const int32_t *col, int32_t n, int32_t *counts, hipStream_t s);
// Pivot at the first maximum of counts[i+1] - counts[i], random permutation
// of each part, riffle. Synchronizes s once (the pivot sizes the parts).
// Workspace: gradient_perm_ws_bytes(n).
size_t gradient_perm_ws_bytes(int64_t n);
hipError_t launch_gradient_perm(int64_t n, const int32_t *counts, uint64_t stream_seed,
                                int32_t *perm, int32_t *inv, void *ws, hipStream_t s);

// ---- permuted CSR --------------------------------------------------------
// rp_b[i'] = exclusive prefix of A's row lengths taken in rperm order.
// Workspace: permuted_row_ptr_ws_bytes(nrows).
size_t permuted_row_ptr_ws_bytes(int32_t nrows);
hipError_t launch_permuted_row_ptr(int32_t nrows, const int32_t *rp, const int32_t *rperm,
                                   int32_t *rp_b, void *ws, hipStream_t s);
// Row i of A -> row rinv[i] of B (at rp_b[rinv[i]]) with column j -> cinv[j]
// (cinv may be NULL: no column permutation), re-sorted by new column.
// val_bytes: 8, 4, 2.
hipError_t launch_gather_relabel_sort(int32_t nrows, const int32_t *rp, const int32_t *col,
                                      const void *val, int val_bytes, const int32_t *rinv,
                                      const int32_t *cinv, const int32_t *rp_b, int32_t *col_b,
                                      void *val_b, hipStream_t s);

// ---- vectors --------------------------------------------------------------
// elem_bytes 8 (FP64) or 4 (FP32).
hipError_t launch_gather_rows(int32_t n, int32_t k, const int32_t *perm, const void *X,
                              int64_t ldx, void *Xp, int64_t ldxp, int elem_bytes, hipStream_t s);
hipError_t launch_scatter_rows(int32_t n, int32_t k, const int32_t *perm, const void *Yp,
                               int64_t ldyp, void *Y, int64_t ldy, int elem_bytes, hipStream_t s);

// ---- values ----------------------------------------------------------------
hipError_t launch_convert_f64(const double *in, void *out, int64_t n, int dtype, hipStream_t s);

// ---- row statistics and length bins --------------------------------------
constexpr int kNumBins = 7;              // lanes per row 1, 2, 4, ..., 64
// Writes the longest row length to *max_len (device int32).
hipError_t launch_row_max(int32_t nrows, const int32_t *rp, int32_t *max_len, hipStream_t s);
// Stable partition of the rows by length bin: rows with bin b fill
// list[bin_off[b] .. bin_off[b+1]) in increasing order. bin_off (device,
// kNumBins + 1 int32). Workspace: row_bins_ws_bytes(nrows).
size_t row_bins_ws_bytes(int32_t nrows);
hipError_t launch_row_bins(int32_t nrows, const int32_t *rp, int32_t *list, int32_t *bin_off,
                           void *ws, hipStream_t s);
// lanes for a row of length len in the binned variant
__host__ __device__ inline int bin_of_length(int32_t len) {
    int b = 0;
    while (b < kNumBins - 1 && len > (2 << b)) ++b;   // <=2: 1 lane, <=4: 2, ..., >64: 64
    return b;
}

// ---- histogram and entropy -------------------------------------------------
// hist: grid_r * grid_c uint32 (device). Workspace: block_hist_ws_bytes().
hipError_t launch_block_hist(int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *rp,
                             const int32_t *col, int32_t grid_r, int32_t grid_c, uint32_t *hist,
                             hipStream_t s);
// result (device, 4 doubles): h_bits, h_nats, certified (1.0 / 0.0), S.
size_t entropy_ws_bytes(int64_t bins);
hipError_t launch_entropy(const uint32_t *hist, int64_t bins, double *result, void *ws,
                          hipStream_t s);
// Hierarchical entropy: for each level L, min(L, G_r) x min(L, G_c) regions;
// result holds 4 doubles per region (as launch_entropy), levels in order,
// regions row-major. Synchronizes s (the region table is staged from the host).
int32_t entropy_regions_count(int32_t grid_r, int32_t grid_c, const int32_t *levels,
                              int32_t nlevels);
size_t entropy_regions_ws_bytes(int32_t grid_r, int32_t grid_c, const int32_t *levels,
                                int32_t nlevels);
hipError_t launch_entropy_regions(const uint32_t *hist, int32_t grid_r, int32_t grid_c,
                                  const int32_t *levels, int32_t nlevels, double *result,
                                  void *ws, hipStream_t s);

// ---- SpMV / SpMM ------------------------------------------------------------
enum ValType { VAL_F64 = 0, VAL_F32 = 1, VAL_BF16 = 2 };

// Column-slab layout (kernels_slab.hip): geometry for one right-hand-side class.
struct SlabGeom {
    int32_t nrows, ncols;
    int32_t slabs, width, cbits;          // column slabs of `width` columns
    int32_t rows_per_block, rows_per_sub; // workgroup block, wavefront sub-block
    int32_t blocks, kclass;
};
// cu_count: the CUs the row blocks are sized for (two blocks each);
// y_lds_bytes: the LDS a block's partial y may take; resident: the blocks
// that run at once, in whose whole waves rows are spread when y_lds_bytes
// caps the blocks (0: blocks of the capped size, for the batch's work
// queues). false when the matrix cannot use the layout (packed indices would
// not fit)
bool slab_geometry(int32_t nrows, int32_t ncols, int kclass, int vtype, int cu_count,
                   int64_t slab_bytes, int64_t y_lds_bytes, int64_t resident, SlabGeom *g);
size_t slab_offsets_count(const SlabGeom &g);
size_t slab_build_ws_bytes(const SlabGeom &g);
hipError_t launch_slab_build(const SlabGeom &g, const int32_t *rp, const int32_t *col,
                             const void *val, int val_bytes, int32_t *off, uint32_t *idx_out,
                             void *val_out, void *ws, hipStream_t s);
// Whole X rows may be read as 16-byte vectors when each row is exactly kclass
// values (elem_bytes each) on a 16-byte boundary: never a read past a row's k
// values.
inline bool slab_vec_x(int kclass, int32_t k, const void *X, int64_t ldx, int elem_bytes) {
    // the slab kernel reads an X row min(16, kclass x elem_bytes) bytes at a time
    const int64_t vb = (int64_t)kclass * elem_bytes < 16 ? (int64_t)kclass * elem_bytes : 16;
    return kclass > 1 && k == kclass && (ldx * elem_bytes) % vb == 0 &&
           (reinterpret_cast<uintptr_t>(X) % vb) == 0;
}
// The x window of MXE_VAR_WINDOW: in a block's dynamic LDS, after its partial
// y (rows_per_block x kclass values of elem_bytes), 16-byte aligned.
__host__ __device__ inline size_t slab_window_offset(const SlabGeom &g, int elem_bytes) {
    return ((size_t)g.rows_per_block * g.kclass * elem_bytes + 15) / 16 * 16;
}
// wstart (device, g.blocks int32): each block's window start for windows of
// win columns (x rows).
hipError_t launch_slab_window(const SlabGeom &g, const int32_t *rp, const int32_t *col, int32_t win,
                              int32_t *wstart, hipStream_t s);
// semiring: MXE_SR_* (mxe.h). win > 0 (plus semiring (+, *)): each block
// reads x rows [wstart[b], wstart[b] + win) from an LDS copy (MXE_VAR_WINDOW);
// the dynamic LDS then grows by win x kclass values.
hipError_t launch_spmv_slab(const SlabGeom &g, int vtype, int semiring, const int32_t *off,
                            const uint32_t *idx, const void *val, int32_t k, const void *X,
                            int64_t ldx, void *Y, int64_t ldy, const int32_t *wstart, int32_t win,
                            hipStream_t s);

struct SpmvArgs {
    int32_t nrows, ncols;
    int64_t nnz;
    const int32_t *rp, *col;
    const void *val;
    int vtype;                 // ValType; X/Y are FP64 for VAL_F64 else FP32
    int32_t k;
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    // binned variant
    const int32_t *bin_list;
    const int32_t *bin_off_host;   // kNumBins + 1 host ints
    // merge variant: the matrix's slice starts (merge_coords_bytes, built once
    // by launch_merge_coords, read only)
    const void *merge_coords;
    // MERGE / COO: this launch's own carry workspace (merge_carry_bytes /
    // coo_ws_bytes); never shared between launches that may overlap
    void *carry_ws;
    // slab variant layout (null when not built)
    const SlabGeom *slab;
    const int32_t *slab_off;
    const uint32_t *slab_idx;
    const void *slab_val;
    // window variant: per-block window starts and the window's rows of x
    const int32_t *slab_wstart;
    int32_t slab_win;
    // COO variant: row index per entry (built once, read only)
    const int32_t *coo_row;
};

size_t merge_coords_bytes(int32_t nrows, int64_t nnz);
size_t merge_carry_bytes(int32_t nrows, int64_t nnz);
hipError_t launch_merge_coords(int32_t nrows, int64_t nnz, const int32_t *rp, void *coords,
                               hipStream_t s);
// Y = M X over MXE_SR_MIN_PLUS or MXE_SR_OR_AND (mxe.h), k <= 16.
hipError_t launch_spmv_semiring(const SpmvArgs &a, int semiring, hipStream_t s);
// one COO launch's carries for k class kclass and elem_bytes-wide sums
size_t coo_ws_bytes(int64_t nnz, int kclass, int elem_bytes);
hipError_t launch_coo_rows(int32_t nrows, const int32_t *rp, int32_t *row, hipStream_t s);
// variant: MXE_VARIANT(family, lanes) as in mxe.h
hipError_t launch_spmv(const SpmvArgs &a, int variant, hipStream_t s);

// ---- batched persistent SpMV ------------------------------------------------
struct BatchDesc {             // one piece of one batch item (device-resident table)
    const int32_t *rp, *col;
    const void *val;
    const void *X;
    void *Y;
    int64_t ldx, ldy;
    int32_t nrows, k;
    int32_t vtype;             // ValType
    int32_t kclass;            // k rounded up to a power of two
    int32_t lanes;             // row tiles: lanes per row (1..64), >= kclass
    int32_t rows_per_tile;     // row tiles: rows one work unit covers
    int32_t tile_begin;        // first work unit of this piece within its queue
    int32_t unit0, units;      // the piece: the item's work units [unit0, unit0 + units)
    int32_t item;              // index of the item in the batch
    // per-column outputs (null: column q goes to Y + q with ldy): column q of
    // the result goes to ycol[q] (its row 0) with leading dimension ycol_ld[q],
    // so one product can serve several requests' Y (device arrays of k)
    void *const *ycol;
    const int64_t *ycol_ld;
    int32_t vec_x;             // slab units: whole X rows as vector loads (slab_vec_x)
    // slab units (slab_off non-null): one work unit per block of this layout
    // for k class kclass, in place of row tiles
    SlabGeom slab;
    const int32_t *slab_off;
    const uint32_t *slab_idx;
    const void *slab_val;
};
// One work queue per XCD: queue q holds the pieces qent[qbegin[q] ..
// qbegin[q+1]) (indices into the desc table, in unit order) and qtiles[q]
// work units in all.
constexpr int kBatchQueues = 8;
// An item moving more than 1/kBatchQueues of a batch's bytes is cut into
// pieces of at most 1/(2 kBatchQueues) of them, so a batch of n items has at
// most n + 2 kBatchQueues pieces.
constexpr int kBatchExtraPieces = 2 * kBatchQueues;
struct BatchQueues {
    int32_t qbegin[kBatchQueues + 1];
    int32_t qtiles[kBatchQueues];
};
constexpr int kBatchBlock = 1024;       // threads per workgroup of the batch kernel
// counters: kBatchQueues device ints zeroed by launch_batch_reset before each
// launch.
hipError_t launch_batch_reset(int32_t *counters, hipStream_t s);
// Workgroups of the batch kernel resident at once on the current device for
// vtype (a ValType, or -1 for a mixed batch) and lds_bytes of dynamic LDS (the
// largest slab block's partial y); 0 when the query fails. Not a stream
// operation: call it before a graph capture.
int32_t batch_grid_size(int vtype, size_t lds_bytes);
hipError_t launch_spmv_batch(const BatchDesc *descs, const int32_t *qent, const BatchQueues &queues,
                             int32_t *counters, int32_t grid, size_t lds_bytes, int vtype,
                             hipStream_t s);

// ---- random-gather rate probe -------------------------------------------------
// ws: probe_gather_ws_bytes; the table is ws's first table_bytes (8-byte
// values, any contents). Issues probe_gathers_issued(gathers, grid) gathers.
size_t probe_gather_ws_bytes(int64_t table_bytes, int32_t grid);
hipError_t launch_probe_gather(int64_t table_bytes, int64_t gathers, int per_xcd, void *ws,
                               int32_t grid, hipStream_t s);
int64_t probe_gathers_issued(int64_t gathers, int32_t grid);

// ---- serving: pack / unpack merged right-hand sides -------------------------
// Copies k columns between a caller matrix (ld) and columns [c0, c0+k) of a
// packed matrix (ldp); elem_bytes 8 or 4.
hipError_t launch_copy_cols(int32_t n, int32_t k, const void *src, int64_t lds, void *dst,
                            int64_t ldd, int elem_bytes, hipStream_t s);
// One column block of a packed matrix: rows [0, n) of src (k columns, leading
// dimension lds) go to columns [c0, c0 + k) of dst (leading dimension ldd).
struct PackCols {
    const void *src;
    int64_t lds;
    void *dst;
    int64_t ldd;
    int32_t n, k, c0, pad;
};
// count entries of a device table, at once; max_n: the largest n among them.
hipError_t launch_pack_cols(const PackCols *table, int32_t count, int32_t max_n, int elem_bytes,
                            hipStream_t s);

}  // namespace mxe
