"""Host-side checks of the benchmark scripts' contract (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_algorithmic_bytes_of_the_n2m_fp64_product():
    import bench
    # nnz (8-byte value + 4-byte column) + (M + 1) row pointers + x and y once, FP64
    n, nnz = 2_000_000, 20_000_000
    assert bench.spmv_bytes(n, n, nnz, 8, 8) == nnz * 12 + (n + 1) * 4 + 2 * n * 8 == 280_000_004


def test_extras_rejects_unknown_parts():
    import bench_extras
    with pytest.raises(SystemExit) as e:
        bench_extras.main(["no_such_part"])
    assert e.value.code == 2
    assert set(bench_extras.PARTS) == {"skewed", "heavy", "semiring", "batch", "serving"}
