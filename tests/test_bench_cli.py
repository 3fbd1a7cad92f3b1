"""bench.py's command line on the host: one GPU only, known workloads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_workload_is_refused():
    r = run("--workload", "nonexistent")
    assert r.returncode != 0


def test_byte_model_of_the_dominant_kernels():
    sys.path.insert(0, ROOT)
    import bench
    n, m = 1 << 20, 1 << 24
    # first pass: CSR destinations + offsets in, key32 + source out
    assert bench.kernel_bytes("k_lsd_pass0", n, m, 0, 2) == 4 * m + 8 * (n + 1) + 8 * m
    # last pass with payload: key32 + source + payload in, key16 + source + payload out
    assert bench.kernel_bytes("k_lsd_pass1", n, m, 4, 2) == 12 * m + 10 * m
    # packed intermediate of a two-pass plan: 16-bit key + source word between the passes
    assert bench.kernel_bytes("k_lsd_pass0", n, m, 0, 2, packed=True) == 4 * m + 8 * (n + 1) + 6 * m
    assert bench.kernel_bytes("k_lsd_pass1", n, m, 4, 2, packed=True) == 10 * m + 10 * m
    assert bench.kernel_bytes("k_final", n, m, 0, 2) == 6 * m + 4 * m + 8 * (n + 1)
    # a later pass's tile counts: one read of its input keys
    assert bench.kernel_bytes("k_tile_hist", n, m, 0, 2, packed=True) == 2 * m
    assert bench.kernel_bytes("k_tile_hist", n, m, 4, 3) == 4 * m
    assert bench.path_alg_bytes(n, m, 0) == 2 * (8 * (n + 1) + 4 * m) + 8 * n


def test_microbench_levels_and_gpu_requirement():
    import torch
    from paper_2501_06872_amd import microbench as mb
    # every level fits the limits of the entry point
    for name, (memory, words) in mb.LEVELS.items():
        assert 1 <= words <= (16384 if memory == 1 else 1 << 32), name
    if not torch.cuda.is_available():
        with pytest.raises(SystemExit):
            mb.main([])
