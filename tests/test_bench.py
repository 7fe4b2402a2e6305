"""Host-side arithmetic of the benchmark line: the compulsory HBM bytes that
price the roofline, and the paper-style logical bytes per nonzero, against
hand counts for the 4-mode and 5-mode skewed tensors."""
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import bench  # noqa: E402


def test_compulsory_bytes_of_the_4_mode_tensor():
    # 145 190 717 nonzeros x (8-byte index + 4-byte value), the other modes'
    # rows once (R = 32 FP32: 128 B each), the output rows once in FP32
    info = {"dims": [1_000_000, 100_000, 10_000, 500], "nnz": 145_190_717, "key_bits": 64}
    assert bench.compulsory_bytes(info, 32, 4, 0) == 145_190_717 * 12 + (100_000 + 10_000 + 500) * 128 + 1_000_000 * 128
    assert bench.compulsory_bytes(info, 32, 4, 0) == 1_884_432_604
    # BF16 factors halve the gathered rows, not the FP32 output
    assert bench.compulsory_bytes(info, 32, 2, 3) == 145_190_717 * 12 + (1_000_000 + 100_000 + 10_000) * 64 + 500 * 128
    # at 8 TB/s the floor is 0.236 ms per launch
    assert bench.compulsory_bytes(info, 32, 4, 0) / 8e12 == pytest.approx(0.2356e-3, rel=1e-3)


def test_compulsory_bytes_of_the_5_mode_tensor():
    # 128-bit index: 16 + 4 bytes per nonzero
    dims = [10_000_000, 5_000_000, 2_000_000, 100_000, 1_000]
    info = {"dims": dims, "nnz": 199_704_254, "key_bits": 128}
    for mode in range(5):
        want = 199_704_254 * 20 + sum(d * 128 for m, d in enumerate(dims) if m != mode) + dims[mode] * 128
        assert bench.compulsory_bytes(info, 32, 4, mode) == want
    assert bench.compulsory_bytes(info, 32, 4, 0) == 6_183_013_080


def test_logical_bytes_per_nonzero():
    # W/8 + 4 + (N-1) R s_f + 4R: 524 B (FP32) and 332 B (BF16) on the 4-mode
    # tensor, 660 B and 404 B on the 5-mode one, 204 B at R = 16 on the 3-mode one
    assert bench.logical_bytes_per_nnz(4, 32, 64, 4) == 524
    assert bench.logical_bytes_per_nnz(4, 32, 64, 2) == 332
    assert bench.logical_bytes_per_nnz(5, 32, 128, 4) == 660
    assert bench.logical_bytes_per_nnz(5, 32, 128, 2) == 404
    assert bench.logical_bytes_per_nnz(3, 16, 64, 4) == 204
