"""ORACLE — test infrastructure only (see oracle/__init__.py).

Degree sampling and graph features, written out plainly in numpy/fp64 from
their definition (Section IV-C, Step 0: a sample of 1% of |V| positions of the
edge array; Section V-G: coverage of the most frequent destinations).

Sample i of s takes position lo + (r mod (hi - lo)) in the stratum
[lo, hi) = [floor(i m / s), floor((i+1) m / s)), r being the (i+1)-th output of
splitmix64 seeded with `seed` (Steele, Lea, Flood 2014).
"""
import math

import numpy as np

NUM_FEATURES = 16
BIG_BIN_EDGES = 8192.0
MASK64 = (1 << 64) - 1


def splitmix64(seed, i):
    """(i+1)-th output of splitmix64 seeded with `seed` (Python integers)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_np(seed, i):
    """Vectorised splitmix64 (numpy uint64 wraps modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (i.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sample_count(n, m):
    s = max((n + 99) // 100, 4096)
    return min(s, m)


def sample_positions(n, m, seed):
    s = sample_count(n, m)
    i = np.arange(s, dtype=np.uint64)
    q, r = np.uint64(m // s), np.uint64(m % s)
    lo = i * q + (i * r) // np.uint64(s)
    hi = (i + np.uint64(1)) * q + ((i + np.uint64(1)) * r) // np.uint64(s)
    return lo + splitmix64_np(seed, i) % (hi - lo)


def features(O, D, payload, seed):
    """The feature vector (float32[16]) the plan computes for this graph."""
    O = np.asarray(O, dtype=np.int64)
    D = np.asarray(D, dtype=np.int32)
    n, m = O.size - 1, D.size
    f = np.zeros(NUM_FEATURES, dtype=np.float64)
    f[0] = math.log2(n + 1.0) / 32.0
    f[1] = math.log2(m + 1.0) / 40.0
    f[2] = math.log2(m / (n if n > 0 else 1.0) + 1.0) / 8.0
    f[3] = 1.0 if payload else 0.0
    if n == 0 or m == 0:
        return f.astype(np.float32)
    s = sample_count(n, m)
    pos = sample_positions(n, m, seed).astype(np.int64)
    dst = D[pos].astype(np.int64)
    dst[(dst < 0) | (dst >= n)] = 0
    src = np.searchsorted(O, pos, side="right") - 1          # largest u with O[u] <= pos
    keys, counts = np.unique(dst, return_counts=True)
    bucket = np.array([int(c).bit_length() - 1 for c in counts], dtype=np.int64)
    nkeys = np.bincount(bucket, minlength=32).astype(np.float64)
    sums = np.bincount(bucket, weights=counts.astype(np.float64), minlength=32)
    for t, j0 in enumerate((1, 2, 4, 6)):
        f[4 + t] = sums[j0:].sum() / s
    for t, lk in enumerate((10, 14, 18)):
        need, cov = float(1 << lk), 0.0
        for j in range(31, -1, -1):
            if need <= 0:
                break
            if nkeys[j] <= 0:
                continue
            if nkeys[j] <= need:
                cov += sums[j]
                need -= nkeys[j]
            else:
                cov += need * (sums[j] / nkeys[j])
                need = 0.0
        f[8 + t] = cov / s
    dist = np.abs(dst - src)
    f[11] = float(dist.sum()) / (s * float(n))
    f[12] = np.count_nonzero(dist < 256) / s
    f[13] = np.count_nonzero(dist < 65536) / s
    binc = np.bincount(dst >> 8)
    scale = m / s
    f[14] = float(binc[binc.astype(np.float64) * scale > BIG_BIN_EDGES].sum()) / s
    f[15] = keys.size / s
    return f.astype(np.float32)
