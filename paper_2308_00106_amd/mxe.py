"""ctypes binding of libmxe.so (include/mxe.h). Argument marshalling only:
every step runs in the library's HIP kernels. torch supplies device memory
(tensor.data_ptr()) and streams (torch.cuda.Stream.cuda_stream).

Names follow the C ABI without the `mxe_` prefix. Loading fails loudly if the
library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmxe.so")

# status codes
OK, ERR_INVALID_ARG, ERR_INVALID_CSR, ERR_NOT_FOUND, ERR_BUSY, ERR_BUDGET = 0, 1, 2, 3, 4, 5
ERR_OUT_OF_MEMORY, ERR_UNSUPPORTED, ERR_TIMEOUT, ERR_DEVICE, ERR_INEXACT = 6, 7, 8, 9, 10
# storage dtypes
F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
# flags
INPUT_DEVICE = OUTPUT_DEVICE = 0x1
ROWS, COLS, GRADIENT = 0x1, 0x2, 0x4
SPACE_PERMUTED, SPACE_ORIGINAL = 0x0, 0x1
VAR_GROUP, VAR_BINNED, VAR_MERGE, VAR_SLAB, VAR_FIXED, VAR_COO = 0x000, 0x100, 0x200, 0x300, 0x400, 0x500
VAR_WINDOW = 0x600                # SLAB layout plus an LDS window of x per row block
SLAB_ONE_PER_CU = 0x80            # SLAB lanes flag: row blocks for one workgroup per CU
SR_PLUS_TIMES, SR_MIN_PLUS, SR_OR_AND = 0, 1, 2
# allocation-free batches: items per call, bytes of the static device scratch array
NOALLOC_MAX_ITEMS, NOALLOC_SCRATCH_BYTES = 256, 65536
SERVE_MAX_BATCH = 64              # requests per serving launch, at most


def variant(family: int, lanes: int = 0) -> int:
    return family | lanes


class MxeError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        super().__init__(f"{func}: {status_string(status)} ({status}): {detail}")


class _Item(ctypes.Structure):
    _fields_ = [("mat", ctypes.c_int64), ("k", ctypes.c_int32), ("X", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64),
                ("flags", ctypes.c_uint32)]


class _Desc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("storage", ctypes.c_int32), ("permuted", ctypes.c_int32),
                ("parent", ctypes.c_int64), ("seed", ctypes.c_uint64), ("mode", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64), ("max_row", ctypes.c_int32),
                ("mean_row", ctypes.c_double)]


class _ServeCfg(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_merge_k", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libmxe.so (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2308_00106_amd.build`")
    # torch first: its wheel carries its own HIP runtime under the same soname,
    # so libmxe.so then binds to the copy torch already loaded and both share
    # one runtime. Loaded the other way round, a second runtime comes in from
    # the system and torch afterwards finds no GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    st = ctypes.c_int
    sigs = {
        "mxe_status_string": ([st], ctypes.c_char_p),
        "mxe_last_error": ([], ctypes.c_char_p),
        "mxe_abi_version": ([], i32),
        "mxe_create": ([i32, u64, P], st),
        "mxe_destroy": ([P], st),
        "mxe_validate_csr": ([i32, i32, i64, P, P], st),
        "mxe_register_matrix": ([P, i32, i32, i64, P, P, P, st, u32, P], st),
        "mxe_permute": ([P, i64, u64, u32, P, P], st),
        "mxe_get_permutation": ([P, i64, P, P, u32, P], st),
        "mxe_export_csr": ([P, i64, P, P, P, u32, P], st),
        "mxe_matrix_info": ([P, i64, P], st),
        "mxe_release": ([P, i64], st),
        "mxe_entropy": ([P, i64, i32, i32, P, P, P, P], st),
        "mxe_entropy_levels": ([P, i64, i32, i32, P, i32, P, P, P], st),
        "mxe_spmv": ([P, i64, i32, P, i64, P, i64, u32, P], st),
        "mxe_gather_x": ([P, i64, i32, P, i64, P, i64, P], st),
        "mxe_scatter_y": ([P, i64, i32, P, i64, P, i64, P], st),
        "mxe_tune": ([P, i64, i32, P, P], st),
        "mxe_set_variant": ([P, i64, i32, i32], st),
        "mxe_probe_gather": ([P, i64, i64, i32, P, P], st),
        "mxe_spmv_semiring": ([P, i64, i32, i32, P, i64, P, i64, u32, P], st),
        "mxe_spmv_batch": ([P, i32, P, P], st),
        "mxe_spmv_batch_noalloc": ([P, i32, P, P], st),
        "mxe_batch_create": ([P, i32, P, P], st),
        "mxe_batch_launch": ([P, i64, P, P], st),
        "mxe_batch_destroy": ([P, i64], st),
        "mxe_serve_start": ([P, P], st),
        "mxe_submit": ([P, P, P], st),
        "mxe_wait": ([P, i64, i64, P], st),
        "mxe_serve_stop": ([P], st),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return [n for n in dir(load_library()) if n.startswith("mxe_")]


def status_string(s: int) -> str:
    return load_library().mxe_status_string(s).decode()


def last_error() -> str:
    return load_library().mxe_last_error().decode()


def abi_version() -> int:
    return int(load_library().mxe_abi_version())


def _check(status: int, func: str) -> None:
    if status != OK:
        raise MxeError(status, func, last_error())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def validate_csr(nrows: int, ncols: int, row_ptr, col_idx) -> int:
    """Returns the status of the host-side canonical-CSR check (no device)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    nnz = int(rp[-1]) if len(rp) == nrows + 1 else len(ci)
    if len(rp) != nrows + 1:
        return ERR_INVALID_ARG
    if len(ci) != nnz:
        return ERR_INVALID_CSR
    return int(load_library().mxe_validate_csr(nrows, ncols, nnz, _np_ptr(rp),
                                               _np_ptr(ci) if len(ci) else None))


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dense(t, rows: int, fp64: bool, name: str):
    """(pointer, k, ld) of a [rows] or [rows, k] row-major device tensor."""
    import torch
    want = torch.float64 if fp64 else torch.float32
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != want:
        raise ValueError(f"{name} must be {want}, got {t.dtype}")
    if t.dim() == 1:
        if t.shape[0] != rows or (rows > 1 and t.stride(0) != 1):
            raise ValueError(f"{name} must have {rows} contiguous elements")
        return ctypes.c_void_p(t.data_ptr()), 1, 1
    if t.dim() != 2 or t.shape[0] != rows or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be [{rows}, k] with unit column stride")
    k = t.shape[1]
    ld = t.stride(0) if rows > 1 else k
    return ctypes.c_void_p(t.data_ptr()), k, max(ld, k)


@dataclass
class MatrixInfo:
    nrows: int
    ncols: int
    nnz: int
    storage: int
    permuted: bool
    parent: int
    seed: int
    mode: int
    device_bytes: int
    max_row: int
    mean_row: float


class Context:
    """One mxe context (mxe_create / mxe_destroy) on a HIP device."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.mxe_create(device, budget_bytes, ctypes.byref(h)), "mxe_create")
        self._h = h
        self._meta = {}

    def close(self) -> None:
        if self._h:
            _check(self._lib.mxe_destroy(self._h), "mxe_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- matrices ---------------------------------------------------------
    def register_matrix(self, nrows: int, ncols: int, row_ptr, col_idx, vals,
                        storage: str = "f64") -> int:
        """Host numpy arrays or device torch tensors (int32, int32, float64)."""
        st = DTYPES[storage]
        out = ctypes.c_int64()
        if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda:
            nnz = int(col_idx.numel())
            args = [ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col_idx.data_ptr()),
                    ctypes.c_void_p(vals.data_ptr()), st, INPUT_DEVICE]
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            va = np.ascontiguousarray(vals, dtype=np.float64)
            nnz = len(ci)
            args = [_np_ptr(rp), _np_ptr(ci) if nnz else None, _np_ptr(va) if nnz else None, st, 0]
        _check(self._lib.mxe_register_matrix(self._h, nrows, ncols, nnz, *args, ctypes.byref(out)),
               "mxe_register_matrix")
        self._meta[out.value] = (nrows, ncols, storage)
        return out.value

    def register(self, A, storage: str = "f64") -> int:
        """Registers a synth.CSR-like object (nrows, ncols, row_ptr, col, val)."""
        return self.register_matrix(A.nrows, A.ncols, A.row_ptr, A.col, A.val, storage)

    def permute(self, a: int, seed: int, mode: int = ROWS | COLS, stream=None) -> int:
        out = ctypes.c_int64()
        _check(self._lib.mxe_permute(self._h, a, seed & (2**64 - 1), mode, _stream_ptr(stream),
                                     ctypes.byref(out)), "mxe_permute")
        self._meta[out.value] = self._meta[a]
        return out.value

    def get_permutation(self, b: int, stream=None):
        nrows, ncols, _ = self._meta[b]
        rp = np.empty(nrows, np.int32)
        cp = np.empty(ncols, np.int32)
        _check(self._lib.mxe_get_permutation(self._h, b, _np_ptr(rp), _np_ptr(cp), 0,
                                             _stream_ptr(stream)), "mxe_get_permutation")
        return rp, cp

    def export_csr(self, m: int, stream=None):
        info = self.matrix_info(m)
        rp = np.empty(info.nrows + 1, np.int32)
        ci = np.empty(info.nnz, np.int32)
        vt = {F64: np.float64, F32: np.float32, BF16: np.uint16}[info.storage]
        va = np.empty(info.nnz, vt)
        _check(self._lib.mxe_export_csr(self._h, m, _np_ptr(rp), _np_ptr(ci), _np_ptr(va), 0,
                                        _stream_ptr(stream)), "mxe_export_csr")
        return rp, ci, va

    def matrix_info(self, m: int) -> MatrixInfo:
        d = _Desc()
        _check(self._lib.mxe_matrix_info(self._h, m, ctypes.byref(d)), "mxe_matrix_info")
        return MatrixInfo(d.nrows, d.ncols, d.nnz, d.storage, bool(d.permuted), d.parent, d.seed,
                          d.mode, d.device_bytes, d.max_row, d.mean_row)

    def release(self, m: int) -> None:
        _check(self._lib.mxe_release(self._h, m), "mxe_release")
        self._meta.pop(m, None)

    # --- measure ------------------------------------------------------------
    def entropy(self, m: int, grid_rows: int, grid_cols: int, stream=None, hist: bool = False):
        """(h_bits, h_nats) or (h_bits, h_nats, hist[grid_rows, grid_cols] int64)."""
        hb, hn = ctypes.c_double(), ctypes.c_double()
        h = np.empty((grid_rows, grid_cols), np.int64) if hist else None
        _check(self._lib.mxe_entropy(self._h, m, grid_rows, grid_cols, _stream_ptr(stream),
                                     ctypes.byref(hb), ctypes.byref(hn),
                                     _np_ptr(h) if hist else None), "mxe_entropy")
        return (hb.value, hn.value, h) if hist else (hb.value, hn.value)

    def entropy_levels(self, m: int, grid_rows: int, grid_cols: int, levels=(2, 4, 8),
                       stream=None):
        """Hierarchical 2D entropy: a list of (bits, nats) arrays, one
        [min(L, grid_rows), min(L, grid_cols)] pair per level L."""
        lv = np.ascontiguousarray(levels, dtype=np.int32)
        shapes = [(min(L, grid_rows), min(L, grid_cols)) for L in levels]
        n = sum(a * b for a, b in shapes)
        hb = np.empty(n, np.float64)
        hn = np.empty(n, np.float64)
        _check(self._lib.mxe_entropy_levels(self._h, m, grid_rows, grid_cols, _np_ptr(lv), len(lv),
                                            _stream_ptr(stream), _np_ptr(hb), _np_ptr(hn)),
               "mxe_entropy_levels")
        out, o = [], 0
        for a, b in shapes:
            out.append((hb[o:o + a * b].reshape(a, b), hn[o:o + a * b].reshape(a, b)))
            o += a * b
        return out

    # --- products -------------------------------------------------------------
    def _fp64(self, m: int) -> bool:
        return self._meta[m][2] == "f64"

    def spmv(self, m: int, X, Y, flags: int = SPACE_PERMUTED, stream=None) -> None:
        nrows, ncols, _ = self._meta[m]
        xp, kx, ldx = _dense(X, ncols, self._fp64(m), "X")
        yp, ky, ldy = _dense(Y, nrows, self._fp64(m), "Y")
        if kx != ky:
            raise ValueError("X and Y must have the same number of columns")
        _check(self._lib.mxe_spmv(self._h, m, kx, xp, ldx, yp, ldy, flags, _stream_ptr(stream)),
               "mxe_spmv")

    def spmv_semiring(self, m: int, semiring: int, X, Y, flags: int = SPACE_PERMUTED,
                      stream=None) -> None:
        """Y = M X over SR_MIN_PLUS or SR_OR_AND (SR_PLUS_TIMES is spmv)."""
        nrows, ncols, _ = self._meta[m]
        xp, kx, ldx = _dense(X, ncols, self._fp64(m), "X")
        yp, ky, ldy = _dense(Y, nrows, self._fp64(m), "Y")
        if kx != ky:
            raise ValueError("X and Y must have the same number of columns")
        _check(self._lib.mxe_spmv_semiring(self._h, m, semiring, kx, xp, ldx, yp, ldy, flags,
                                           _stream_ptr(stream)), "mxe_spmv_semiring")

    def gather_x(self, b: int, X, Xp, stream=None) -> None:
        _, ncols, _ = self._meta[b]
        xp, k, ldx = _dense(X, ncols, self._fp64(b), "X")
        pp, k2, ldp = _dense(Xp, ncols, self._fp64(b), "Xp")
        if k != k2:
            raise ValueError("column counts differ")
        _check(self._lib.mxe_gather_x(self._h, b, k, xp, ldx, pp, ldp, _stream_ptr(stream)),
               "mxe_gather_x")

    def scatter_y(self, b: int, Yp, Y, stream=None) -> None:
        nrows, _, _ = self._meta[b]
        pp, k, ldp = _dense(Yp, nrows, self._fp64(b), "Yp")
        yp, k2, ldy = _dense(Y, nrows, self._fp64(b), "Y")
        if k != k2:
            raise ValueError("column counts differ")
        _check(self._lib.mxe_scatter_y(self._h, b, k, pp, ldp, yp, ldy, _stream_ptr(stream)),
               "mxe_scatter_y")

    def tune(self, m: int, k: int = 1, stream=None) -> int:
        v = ctypes.c_int32()
        _check(self._lib.mxe_tune(self._h, m, k, _stream_ptr(stream), ctypes.byref(v)), "mxe_tune")
        return v.value

    def probe_gather(self, table_bytes: int, gathers: int, per_xcd: bool = False,
                     stream=None) -> float:
        """Random 8-byte gathers per second from a table of table_bytes."""
        rate = ctypes.c_double()
        _check(self._lib.mxe_probe_gather(self._h, table_bytes, gathers, int(per_xcd),
                                          _stream_ptr(stream), ctypes.byref(rate)),
               "mxe_probe_gather")
        return rate.value

    def set_variant(self, m: int, k: int, var: int) -> None:
        _check(self._lib.mxe_set_variant(self._h, m, k, var), "mxe_set_variant")

    # --- batches -------------------------------------------------------------------
    def _items(self, items):
        arr = (_Item * len(items))()
        for i, (m, X, Y) in enumerate(items):
            nrows, ncols, _ = self._meta[m]
            xp, k, ldx = _dense(X, ncols, self._fp64(m), "X")
            yp, k2, ldy = _dense(Y, nrows, self._fp64(m), "Y")
            if k != k2:
                raise ValueError("X and Y must have the same number of columns")
            arr[i] = _Item(m, k, xp.value, ldx, yp.value, ldy, SPACE_PERMUTED)
        return arr

    def spmv_batch(self, items, stream=None) -> None:
        """items: list of (matrix, X, Y)."""
        arr = self._items(items)
        _check(self._lib.mxe_spmv_batch(self._h, len(items), arr, _stream_ptr(stream)),
               "mxe_spmv_batch")

    def spmv_batch_noalloc(self, items, stream=None) -> None:
        """items: list of (matrix, X, Y), each matrix already prepared for its
        k by spmv_batch or batch_create; allocates no device memory."""
        arr = self._items(items)
        _check(self._lib.mxe_spmv_batch_noalloc(self._h, len(items), arr, _stream_ptr(stream)),
               "mxe_spmv_batch_noalloc")

    def batch_create(self, items) -> int:
        arr = self._items(items)
        out = ctypes.c_int64()
        _check(self._lib.mxe_batch_create(self._h, len(items), arr, ctypes.byref(out)),
               "mxe_batch_create")
        return out.value

    def batch_launch(self, plan: int, items=None, stream=None) -> None:
        arr = self._items(items) if items is not None else None
        _check(self._lib.mxe_batch_launch(self._h, plan, arr, _stream_ptr(stream)),
               "mxe_batch_launch")

    def batch_destroy(self, plan: int) -> None:
        _check(self._lib.mxe_batch_destroy(self._h, plan), "mxe_batch_destroy")

    # --- serving -------------------------------------------------------------------
    def serve_start(self, streams: int = 2, max_inflight: int = 32, max_batch: int = 8,
                    max_merge_k: int = 8) -> None:
        """max_inflight: products on the device at once; max_batch: items per
        persistent launch; max_merge_k: right-hand sides of a merged item (1
        and 1: each request its own product)."""
        cfg = _ServeCfg(streams, max_inflight, max_batch, max_merge_k)
        _check(self._lib.mxe_serve_start(self._h, ctypes.byref(cfg)), "mxe_serve_start")

    def submit(self, m: int, X, Y, flags: int = SPACE_PERMUTED) -> int:
        nrows, ncols, _ = self._meta[m]
        xp, k, ldx = _dense(X, ncols, self._fp64(m), "X")
        yp, k2, ldy = _dense(Y, nrows, self._fp64(m), "Y")
        if k != k2:
            raise ValueError("X and Y must have the same number of columns")
        it = _Item(m, k, xp.value, ldx, yp.value, ldy, flags)
        t = ctypes.c_int64()
        _check(self._lib.mxe_submit(self._h, ctypes.byref(it), ctypes.byref(t)), "mxe_submit")
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> float:
        """Blocks until done; returns the latency in microseconds."""
        lat = ctypes.c_double()
        _check(self._lib.mxe_wait(self._h, ticket, timeout_us, ctypes.byref(lat)), "mxe_wait")
        return lat.value

    def serve_stop(self) -> None:
        _check(self._lib.mxe_serve_stop(self._h), "mxe_serve_stop")
