"""CPU checks of bench.py's accounting helpers (no GPU): the search's row
strides, the algorithmic byte split priced by the gather ceiling, and the
recall interpolation."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

from .parity import _layout  # noqa: E402


def test_search_stride_is_the_kernels_layout():
    for raw in [64, 96, 100, 104, 128, 192, 200, 256, 384, 385, 400, 512, 513, 1024, 2304, 4608]:
        assert bench._search_stride(raw) == _layout(raw)[0], raw


def test_row_bytes_per_store():
    assert bench.row_bytes(96, 0) == 384 and bench.row_bytes(96, 1) == 192
    assert bench.row_bytes(100, 2) == 104  # FP8 codes and the FP32 row scale


def test_at95_picks_the_first_point_reaching_the_target():
    pts = [dict(recall=0.90, qps=10.0, L=10), dict(recall=0.949, qps=8.0, L=20),
           dict(recall=0.951, qps=6.0, L=30), dict(recall=0.99, qps=2.0, L=40)]
    best, interp = bench.at95(pts)
    assert best["L"] == 30
    # log-QPS interpolation between the bracketing points, at recall 0.95
    want = np.exp(np.log(8.0) + (0.95 - 0.949) / (0.951 - 0.949) * (np.log(6.0) - np.log(8.0)))
    assert abs(interp - want) < 1e-6 * want


def test_kernel_source_hash_covers_both_files():
    h = bench.kernel_source_sha1()
    assert len(h) == 40 and all(c in "0123456789abcdef" for c in h)
    assert bench.KERNEL_SOURCES == ("search_device.h", "search.hip")
