"""ORACLE — test infrastructure only (see oracle/__init__.py).

Replay, in numpy, of the random-access microbenchmark (the GPU counterpart of
the measurement behind Fig. 3, Section III-B): which indices every thread
visits, and what each access kind leaves in the array and in the per-thread
sink.

* ``fmix32``: the 32-bit finalizer of MurmurHash3 (Appleby).  MurmurHash3_x86_32
  of the empty input with seed s equals fmix32(s), which ties this function to
  that hash's published test vectors.
* Thread t draws r_j = fmix32(fmix32(seed ^ t) + (j + 1) * 0x9E3779B9 mod 2^32)
  for j = 0, 1, ... (SplitMix: a Weyl sequence through a mixer), and access j
  goes to index (r_j * words) >> 32, in [0, words).
* Threads are numbered t = block * 256 + lane.  With the LDS memory, block b
  works on its own image buf[b * words, (b + 1) * words).
"""
import numpy as np

THREADS_PER_BLOCK = 256
WEYL = 0x9E3779B9
READ, WRITE, ATOMIC, INDEX = range(4)
GLOBAL, LDS = range(2)


def fmix32(h):
    """MurmurHash3's 32-bit finalizer on a uint32 array (wraps modulo 2^32)."""
    h = np.asarray(h, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x85EBCA6B)
        h ^= h >> np.uint32(13)
        h *= np.uint32(0xC2B2AE35)
        h ^= h >> np.uint32(16)
    return h


def draws(seed, threads, per_thread):
    """r[t, j] for threads 0..threads-1 and accesses 0..per_thread-1 (uint32)."""
    t = np.arange(threads, dtype=np.uint32)
    start = fmix32(np.uint32(seed) ^ t).astype(np.uint64)
    j = np.arange(1, per_thread + 1, dtype=np.uint64)
    ctr = (start[:, None] + j[None, :] * np.uint64(WEYL)) % np.uint64(1 << 32)
    return fmix32(ctr.astype(np.uint32))


def indices(seed, threads, per_thread, words):
    """The index of every access, int64[threads, per_thread]."""
    r = draws(seed, threads, per_thread).astype(np.uint64)
    return ((r * np.uint64(words)) >> np.uint64(32)).astype(np.int64)


def _one_array(a, idx, t, kind):
    """Apply the accesses idx[k, :] of threads t[k] to array a (a copy is
    returned).  Returns (array, sink, writes) where writes lists the (index,
    value) pairs a WRITE may have left (None for other kinds)."""
    a = a.copy()
    sink = np.zeros(t.size, dtype=np.uint32)
    writes = None
    if kind == READ:
        for k in range(t.size):
            sink[k] = np.bitwise_xor.reduce(a[idx[k]], initial=np.uint32(0))
    elif kind == INDEX:
        for k in range(t.size):
            sink[k] = np.bitwise_xor.reduce(idx[k].astype(np.uint32), initial=np.uint32(0))
    elif kind == ATOMIC:
        with np.errstate(over="ignore"):
            a += np.bincount(idx.ravel(), minlength=a.size).astype(np.uint32)
    else:
        writes = (idx.ravel(), np.repeat(t.astype(np.uint32), idx.shape[1]))
        a[writes[0]] = writes[1]   # one of the outcomes the racing stores allow
    return a, sink, writes


def replay(buf, words, kind, memory, seed, per_thread, blocks):
    """What the benchmark computes.  Returns (array after, sink, writes).
    For WRITE several threads may store to one word, so the array after is
    one of the allowed outcomes and `writes` = (indices, values) of every
    store, for check_writes to judge another outcome."""
    buf = np.asarray(buf, dtype=np.uint32)
    threads = blocks * THREADS_PER_BLOCK
    idx = indices(seed, threads, per_thread, words)
    t = np.arange(threads, dtype=np.int64)
    if memory == GLOBAL:
        return _one_array(buf[:words], idx, t, kind)
    out = buf[:blocks * words].copy()
    sink = np.zeros(threads, dtype=np.uint32)
    w_idx, w_val = [], []
    for b in range(blocks):
        rows = slice(b * THREADS_PER_BLOCK, (b + 1) * THREADS_PER_BLOCK)
        img, s, wr = _one_array(out[b * words:(b + 1) * words], idx[rows], t[rows], kind)
        out[b * words:(b + 1) * words] = img
        sink[rows] = s
        if wr is not None:
            w_idx.append(wr[0] + b * words)
            w_val.append(wr[1])
    writes = (np.concatenate(w_idx), np.concatenate(w_val)) if w_idx else None
    return out, sink, writes


def check_writes(before, after, writes):
    """True iff every word no store reached is unchanged and every word some
    store reached holds a value stored there."""
    before = np.asarray(before, dtype=np.uint32)
    after = np.asarray(after, dtype=np.uint32)
    w_idx, w_val = writes
    touched = np.zeros(before.size, dtype=bool)
    touched[w_idx] = True
    if not np.array_equal(before[~touched], after[~touched]):
        return False
    pairs = np.unique(w_idx.astype(np.uint64) << np.uint64(32) | w_val.astype(np.uint64))
    hit = np.flatnonzero(touched).astype(np.uint64)
    got = hit << np.uint64(32) | after[hit.astype(np.int64)].astype(np.uint64)
    return bool(np.isin(got, pairs).all())
