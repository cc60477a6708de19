"""Host-side logic of bench.py that needs no GPU: the one-GPU rule, the
algorithmic byte counts behind the roofline, and the kernel-source hash that
keeps stored counter figures tied to the sources they were taken with."""
import os
import subprocess
import sys
from types import SimpleNamespace

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_sparse_and_dense():
    n, m, k = 10_000, 8, 20
    sparse = SimpleNamespace(n=n, m=m, nnz=n * m * k, store=0, fmt=0)
    # Bellman: P (value + int32 column per entry), g, V; Phi, pi and g^pi out
    assert bench.per_launch_bytes(sparse, "bellman", False) == n * m * k * 12 + n * m * 8 + n * 8 + n * 20
    # J-apply: P^pi rows, x in, y out (FP32 vectors in mixed mode)
    assert bench.per_launch_bytes(sparse, "japply", True) == n * k * 12 + n * 4 * 2
    # refine mode: the products read the BF16 copy of P^pi
    refine = SimpleNamespace(n=n, m=m, nnz=n * m * k, store=1, fmt=0, refine=1)
    assert bench.per_launch_bytes(refine, "japply", True) == n * k * 6 + n * 4 * 2
    # a refine handle stores BF16 for the products and keeps an FP32 copy, which
    # the Bellman pass and the residuals read
    refine16 = SimpleNamespace(n=n, m=m, nnz=n * m * k, store=2, fmt=0, refine=1)
    assert bench.per_launch_bytes(refine16, "japply", True) == n * k * 6 + n * 4 * 2
    assert bench.per_launch_bytes(refine16, "bellman", True) == n * m * k * 8 + n * m * 8 + n * 8 + n * 20
    assert bench.per_launch_bytes(refine16, "residual", True) == n * k * 8 + n * 24
    assert bench.per_launch_bytes(sparse, "residual", False) == n * k * 12 + n * 24
    dense = SimpleNamespace(n=n, m=4, nnz=n * 4 * n, store=2, fmt=1)  # BF16 rows, no column indices
    assert bench.per_launch_bytes(dense, "bellman", True) == n * 4 * n * 2 + n * 4 * 8 + n * 8 + n * 20
    assert bench.per_launch_bytes(dense, "gram_schmidt", True) is None


def test_kernel_groups_and_source_hash():
    assert bench.kernel_group("persistent", 0) == "persistent"
    assert bench.kernel_group("japply", 0) == "sparse"
    assert bench.kernel_group("bellman", 1) == "dense"
    for g in bench.KERNEL_FILES:
        h = bench.kernel_source_hash(g)
        assert len(h) == 16 and h == bench.kernel_source_hash(g)
    assert len({bench.kernel_source_hash(g) for g in bench.KERNEL_FILES}) == len(bench.KERNEL_FILES)
