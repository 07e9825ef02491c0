"""The C-ABI library loads, exports every entry point include/mxe.h declares,
and its host-side checks behave; no compute calls (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mxe.h")

mx = pytest.importorskip("paper_2308_00106_amd.mxe")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mx.LIB_PATH):
        import paper_2308_00106_amd.build as b
        b.build(force=False)
    return mx.load_library()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mxe_[a-z_]+)\s*\(", text)) - {"mxe_status"})


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mxe_register_matrix", "mxe_permute", "mxe_entropy", "mxe_spmv", "mxe_spmv_batch",
              "mxe_submit", "mxe_wait", "mxe_release", "mxe_create", "mxe_destroy"]:
        assert n in names


def test_binding_constants_match_the_header():
    """Every numeric #define of the header (flags, semirings, variant
    families) has the same value in the binding, under its name without the
    MXE_ prefix."""
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define MXE_([A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|[0-9]+)u?\b", text))
    skip = {"ABI_VERSION"}
    checked = 0
    for name, value in defs.items():
        if name in skip:
            continue
        assert hasattr(mx, name), name
        assert getattr(mx, name) == int(value, 0), (name, value)
        checked += 1
    assert checked >= 15
    # the status and storage enumerations, value by value
    enums = re.findall(r"typedef enum \w*\s*\{(.*?)\}", text, re.S)
    assert len(enums) >= 2
    for enum in enums:
        names = re.findall(r"\bMXE_([A-Z0-9_]+)\s*=\s*([0-9]+)", enum)
        assert names
        for name, value in names:
            assert getattr(mx, name) == int(value), name


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version(lib):
    assert mx.abi_version() == 1
    assert mx.status_string(mx.OK) == "ok"
    assert mx.status_string(mx.ERR_INVALID_CSR) == "invalid CSR"
    assert mx.status_string(mx.ERR_INEXACT)


def _v(nrows, ncols, rp, col):
    return mx.validate_csr(nrows, ncols, np.asarray(rp), np.asarray(col))


def test_validate_accepts_canonical_csr(lib):
    A = synth.clustered_n4096(1)
    assert _v(A.nrows, A.ncols, A.row_ptr, A.col) == mx.OK
    assert _v(0, 0, [0], []) == mx.OK
    assert _v(3, 5, [0, 0, 0, 0], []) == mx.OK           # empty rows


@pytest.mark.parametrize("rp,col,why", [
    ([1, 2], [0, 1], "row_ptr[0] != 0"),
    ([0, 2, 1], [0, 1], "decreasing row_ptr"),
    ([0, 2], [1, 1], "duplicate column"),
    ([0, 2], [2, 1], "unsorted columns"),
    ([0, 1], [5], "column out of range"),
    ([0, 1], [-1], "negative column"),
])
def test_validate_rejects_malformed(lib, rp, col, why):
    nrows = len(rp) - 1
    st = _v(nrows, 4, rp, col)
    assert st == mx.ERR_INVALID_CSR, why
    assert mx.last_error()


def test_validate_rejects_bad_sizes(lib):
    st = lib.mxe_validate_csr(-1, 4, 0, None, None)
    assert st == mx.ERR_INVALID_ARG
    rp = np.array([0, 1], np.int32)
    assert lib.mxe_validate_csr(1, 4, 1, rp.ctypes.data_as(ctypes.c_void_p), None) == mx.ERR_INVALID_ARG


def test_null_context_is_rejected(lib):
    out = ctypes.c_int64()
    assert lib.mxe_permute(None, 1, 0, 3, None, ctypes.byref(out)) == mx.ERR_INVALID_ARG
    assert lib.mxe_spmv(None, 1, 1, None, 1, None, 1, 0, None) == mx.ERR_INVALID_ARG
    assert lib.mxe_create(0, 0, None) == mx.ERR_INVALID_ARG


def test_create_without_device_fails_cleanly(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mx.MxeError) as e:
        mx.Context(0)
    assert e.value.status in (mx.ERR_DEVICE, mx.ERR_INVALID_ARG)


def test_library_shares_torchs_hip_runtime():
    """Loading the library before anything imports torch must still leave one
    HIP runtime in the process (torch's), else torch finds no GPU later."""
    import ast
    import subprocess
    import sys
    code = ("from paper_2308_00106_amd import mxe; mxe.load_library(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       cwd=root)
    assert r.returncode == 0, r.stderr
    libs = ast.literal_eval(r.stdout.strip().splitlines()[-1])
    assert len(libs) == 1 and "torch" in libs[0], libs
