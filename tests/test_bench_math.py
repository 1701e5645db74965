"""The arithmetic behind bench.py's line, on the CPU: compulsory bytes and
flops of the block stencil workload (65,536 rows, 2,451,523 stored entries,
n = 128, FP32), and the error measure."""
import sys
from pathlib import Path

import numpy as np

sys.path.insert(0, str(Path(__file__).resolve().parent.parent))
import bench  # noqa: E402


def test_compulsory_bytes_of_the_stencil_step():
    m = k = 65536
    nnz, n = 2_451_523, 128
    # A once (int32 index + FP32 value per entry, row pointer), B once, C once
    fwd = bench.alg_bytes_forward(m, k, nnz, n, 4, 4, 4)
    assert fwd == nnz * 8 + 4 * (m + 1) + k * n * 4 + m * n * 4 == 86_983_196
    # SDDMM: the pattern and row pointer, dC and B once, dA once
    sdd = bench.alg_bytes_sddmm(m, k, nnz, n, 4, 4, 4)
    assert sdd == nnz * 4 + 4 * (m + 1) + m * n * 4 + k * n * 4 + nnz * 4 == 86_983_196
    # the step's three products: 260.9 MB, and 6 nnz n flops (1.883 GFLOP)
    assert round((2 * fwd + sdd) / 1e6, 1) == 260.9
    assert 6 * nnz * n == 1_882_769_664


def test_rel_err():
    ref = np.array([3.0, 4.0])
    assert bench.rel_err(ref, ref) == 0.0
    assert abs(bench.rel_err(ref + np.array([0.3, 0.4]), ref) - 0.1) < 1e-15
    # a zero reference gives the absolute error
    assert bench.rel_err(np.array([3.0, 4.0]), np.zeros(2)) == 5.0
