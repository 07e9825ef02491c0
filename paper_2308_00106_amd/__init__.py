"""mxe: max-entropy permuted sparse matrix-vector products on MI355X (gfx950).

The library (libmxe.so, HIP kernels behind a C ABI declared in
include/mxe.h) randomly permutes a CSR matrix's rows and columns
(B = P_r A P_c), measures the block-grid nonzero entropy, and multiplies the
resident permuted matrix by dense vectors. This package is its ctypes
binding; see `mxe.Context`.
"""
from .mxe import (  # noqa: F401
    BF16, COLS, F32, F64, GRADIENT, ROWS, SPACE_ORIGINAL, SPACE_PERMUTED, VAR_BINNED, VAR_GROUP,
    VAR_COO, VAR_FIXED, VAR_MERGE, VAR_SLAB, Context, MxeError, abi_version, exported_symbols, last_error, load_library,
    SLAB_ONE_PER_CU, SR_MIN_PLUS, SR_OR_AND, SR_PLUS_TIMES, status_string, validate_csr, variant,
)
