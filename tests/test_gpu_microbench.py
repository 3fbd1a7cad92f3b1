"""GPU: the random-access microbenchmark kernels against the oracle's replay
(oracle/random_access.py).  Reads, index draws and atomic counts are
compared bit-exactly; racing plain writes are checked for validity (every
word holds a value some thread stored there, untouched words unchanged)."""
import sys

import numpy as np
import pytest
import torch

from oracle import random_access as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_case(dev, words, kind, memory, seed, per, blocks, init="ramp"):
    import paper_2501_06872_amd as gt
    say(f"[case] words={words} kind={kind} memory={memory} seed={seed} per_thread={per} blocks={blocks}")
    size = words * (blocks if memory == R.LDS else 1)
    rng = np.random.default_rng(seed)
    host = (rng.integers(0, 1 << 32, size, dtype=np.uint64).astype(np.uint32) if init == "random"
            else np.zeros(size, np.uint32))
    buf = torch.from_numpy(host.view(np.int32).copy()).to(dev)
    sink = torch.full((blocks * R.THREADS_PER_BLOCK,), -1, dtype=torch.int32, device=dev)
    gt.random_access(buf, words, kind, memory, seed, per, blocks, sink)
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.uint32)
    got_sink = sink.cpu().numpy().view(np.uint32)
    want, want_sink, writes = R.replay(host, words, kind, memory, seed, per, blocks)
    assert np.array_equal(got_sink, want_sink), "sink differs"
    if kind == R.WRITE:
        assert R.check_writes(host, got, writes), "a word holds a value no thread stored there"
    else:
        assert np.array_equal(got, want), "array differs"


@pytest.mark.parametrize("kind", [R.READ, R.WRITE, R.ATOMIC, R.INDEX])
@pytest.mark.parametrize("memory", [R.GLOBAL, R.LDS])
def test_kinds_match_replay(hip_device, kind, memory):
    run_case(hip_device, 1000, kind, memory, 17, 64, 4, init="random")
    run_case(hip_device, 777, kind, memory, 123456789, 33, 3, init="random")   # ragged sizes


@pytest.mark.parametrize("memory", [R.GLOBAL, R.LDS])
def test_edge_sizes(hip_device, memory):
    run_case(hip_device, 1, R.ATOMIC, memory, 5, 50, 2)            # every access to one word
    run_case(hip_device, 1, R.WRITE, memory, 5, 50, 2)
    run_case(hip_device, 16384, R.ATOMIC, memory, 6, 40, 2)       # the LDS maximum
    run_case(hip_device, 16384, R.READ, memory, 6, 40, 2, init="random")
    run_case(hip_device, 500, R.READ, memory, 8, 0, 2, init="random")   # no accesses: sink 0


def test_large_global_array(hip_device):
    # 2^26 words (256 MB): sampled check of the atomic counts through the
    # replay of the same indices
    import paper_2501_06872_amd as gt
    words, per, blocks, seed = 1 << 26, 16, 64, 99
    say(f"[case] large words={words} per_thread={per} blocks={blocks}")
    buf = torch.zeros(words, dtype=torch.int32, device=hip_device)
    gt.random_access(buf, words, gt.ACCESS_ATOMIC, gt.MEMORY_GLOBAL, seed, per, blocks)
    torch.cuda.synchronize()
    idx = R.indices(seed, blocks * R.THREADS_PER_BLOCK, per, words).ravel()
    want = np.bincount(idx, minlength=words)
    nz = np.flatnonzero(want)
    got = buf.cpu().numpy()
    assert int(got.sum()) == idx.size
    assert np.array_equal(got[nz], want[nz])


def test_argument_errors(hip_device):
    import paper_2501_06872_amd as gt
    buf = torch.zeros(16, dtype=torch.int32, device=hip_device)
    with pytest.raises(gt.GTError) as e:
        gt._check(gt.lib().gt_random_access(buf.data_ptr(), 0, 0, 0, 1, 1, 1, None, None), "x")
    assert e.value.status == gt.GT_ERR_INVALID_ARGUMENT
    with pytest.raises(gt.GTError) as e:
        gt._check(gt.lib().gt_random_access(buf.data_ptr(), 16385, 0, gt.MEMORY_LDS, 1, 1, 1, None, None), "x")
    assert e.value.status == gt.GT_ERR_UNSUPPORTED
    with pytest.raises(gt.GTError) as e:
        gt._check(gt.lib().gt_random_access(buf.data_ptr(), 16, 4, 0, 1, 1, 1, None, None), "x")
    assert e.value.status == gt.GT_ERR_INVALID_ARGUMENT
