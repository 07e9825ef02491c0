"""Helpers for the GPU parity tests (importable without a GPU)."""
import numpy as np

import oracle

TOL = {"f64": 1e-13, "f32": 1e-5, "bf16": 1e-2}


def torch_vec(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dtype, device="cuda")


def stored_csr(A, storage):
    """A with its values replaced by the FP64 value of what the GPU stores."""
    import synth
    return synth.CSR(A.nrows, A.ncols, A.row_ptr, A.col, oracle.stored_values(A.val, storage))


def expected_export(A, rperm, cperm, storage):
    """Oracle's permuted CSR (row_ptr, col, stored value bits)."""
    rp, col, val = oracle.permute_csr(A, rperm, cperm)
    if storage == "f64":
        return rp, col, val
    if storage == "f32":
        return rp, col, oracle.round_f32(val)
    return rp, col, oracle.round_bf16(val)


def spmv_error(A, X, Y, storage, ref_stored=False):
    """Normalized error of Y against the FP64 oracle: on the original FP64
    values (ref_stored False) or on the stored values (True)."""
    Ay = stored_csr(A, storage) if ref_stored else A
    ref = oracle.spmm(A.nrows, Ay.row_ptr, Ay.col, Ay.val, X)
    return oracle.normalized_error(A.nrows, A.row_ptr, A.col, A.val, X, Y, ref)
