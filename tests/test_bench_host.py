"""Host-side parts of bench.py (no GPU): the one-GPU contract and the byte model."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth import random_sparse  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_compulsory_bytes_model():
    A = random_sparse(300, 200, 0.05, seed=3)
    l = 24
    # index + value per nonzero, 32-bit pointers of the segments, input read once, output written once
    assert bench.spmm_bytes(A, l, trans=False) == A.nnz * 8 + (A.m + 1) * 4 + A.n * l * 4 + A.m * l * 4
    assert bench.spmm_bytes(A, l, trans=True) == A.nnz * 8 + (A.n + 1) * 4 + A.m * l * 4 + A.n * l * 4


def test_row_slice_keeps_the_leading_rows():
    A = random_sparse(300, 200, 0.05, seed=4)
    S = bench.slice_rows(A, 120)
    assert S.m == 120 and S.n == A.n and S.nnz == int(A.row_ptr[120])
    assert np.array_equal(S.row_ptr, A.row_ptr[:121])
    assert np.array_equal(S.col, A.col[:S.nnz]) and np.array_equal(S.val, A.val[:S.nnz])
