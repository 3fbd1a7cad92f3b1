"""Pins of the microbenchmark replay (oracle/random_access.py): the mixer
against MurmurHash3's published vectors, the draw sequence against a
step-by-step generator, the index map's range and uniformity, and invariants
between the access kinds."""
import os

import numpy as np
import pytest

from oracle import random_access as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fmix32_py(h):
    # the finalizer written with Python integers, one step at a time
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    return h ^ (h >> 16)


def test_fmix32_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "murmur3_empty.txt")) if l.strip() and l[0] != "#"]
    seeds = np.array([int(a, 16) for a, _ in rows], dtype=np.uint32)
    assert [int(x) for x in R.fmix32(seeds)] == [int(b, 16) for _, b in rows]


def test_fmix32_is_injective_on_a_block():
    x = np.arange(1 << 22, dtype=np.uint32) * np.uint32(977)
    assert np.unique(R.fmix32(x)).size == x.size


def test_draws_follow_the_incremental_generator():
    # the kernel's form: state = fmix32(seed ^ t), then per access
    # state += 0x9E3779B9 and r = fmix32(state)
    seed, threads, per = 0xC0FFEE, 300, 17
    r = R.draws(seed, threads, per)
    for t in (0, 1, 255, 256, 299):
        state = _fmix32_py(seed ^ t)
        for j in range(per):
            state = (state + R.WEYL) & 0xFFFFFFFF
            assert int(r[t, j]) == _fmix32_py(state)


def test_index_range_and_uniformity():
    idx = R.indices(7, 1024, 1000, 1000)
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx.ravel(), minlength=1000)
    expect = idx.size / 1000
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert abs(chi2 - 999) < 6 * np.sqrt(2 * 999)
    # words = 2^32: the index is the draw itself; words = 1: always 0
    assert np.array_equal(R.indices(3, 8, 5, 1 << 32), R.draws(3, 8, 5).astype(np.int64))
    assert not R.indices(3, 8, 5, 1).any()


@pytest.mark.parametrize("memory", [R.GLOBAL, R.LDS])
def test_kinds_agree_with_each_other(memory):
    words, blocks, per = 777, 3, 40
    size = words * (blocks if memory == R.LDS else 1)
    ramp = np.tile(np.arange(words, dtype=np.uint32), size // words)
    rd, s_read, _ = R.replay(ramp, words, R.READ, memory, 11, per, blocks)
    _, s_index, _ = R.replay(ramp, words, R.INDEX, memory, 11, per, blocks)
    assert np.array_equal(rd, ramp) and np.array_equal(s_read, s_index)   # reads of i at index i
    _, s_zero, _ = R.replay(np.zeros(size, np.uint32), words, R.READ, memory, 11, per, blocks)
    assert not s_zero.any()
    at, s_at, _ = R.replay(np.zeros(size, np.uint32), words, R.ATOMIC, memory, 11, per, blocks)
    assert not s_at.any()
    if memory == R.GLOBAL:
        assert int(at.sum()) == blocks * R.THREADS_PER_BLOCK * per
    else:  # every block's image counts its own 256 threads' accesses
        assert np.all(at.reshape(blocks, words).sum(axis=1) == R.THREADS_PER_BLOCK * per)
    before = np.full(size, 0xFFFFFFFF, np.uint32)
    wr, _, writes = R.replay(before, words, R.WRITE, memory, 11, per, blocks)
    assert R.check_writes(before, wr, writes)


def test_lds_blocks_are_independent_replays():
    # block b of the LDS form replays threads b*256.. on its own image
    words, per = 300, 9
    at, _, _ = R.replay(np.zeros(2 * words, np.uint32), words, R.ATOMIC, R.LDS, 5, per, 2)
    idx = R.indices(5, 512, per, words)
    assert np.array_equal(at[words:], np.bincount(idx[256:].ravel(), minlength=words).astype(np.uint32))


def test_write_check_catches_planted_mistakes():
    words, per = 500, 8
    before = np.zeros(words, np.uint32)
    wr, _, writes = R.replay(before, words, R.WRITE, R.GLOBAL, 2, per, 1)
    assert R.check_writes(before, wr, writes)
    bad = wr.copy()
    hit = int(writes[0][0])
    bad[hit] = 0xDEAD            # a value no thread stored at that index
    assert not R.check_writes(before, bad, writes)
    bad = wr.copy()
    untouched = np.setdiff1d(np.arange(words), writes[0])[0]
    bad[untouched] = 1           # a word no store reached has changed
    assert not R.check_writes(before, bad, writes)
