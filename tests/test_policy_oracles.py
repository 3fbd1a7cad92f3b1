"""Pins of the sampling-feature and MLP oracles (CPU only)."""
import os

import numpy as np
import pytest

from oracle import features as F
from oracle import mlp as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    seed = int(lines[0][1])
    expect = [int(l[0]) for l in lines[1:]]
    assert [F.splitmix64(seed, i) for i in range(3)] == expect
    v = F.splitmix64_np(seed, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in v] == expect


def test_sample_positions_one_per_stratum():
    for n, m in [(10, 50), (1000, 4096), (5000, 123457), (300000, 4800000)]:
        s = F.sample_count(n, m)
        pos = F.sample_positions(n, m, seed=9).astype(np.int64)
        assert pos.size == s
        i = np.arange(s)
        lo = (i * m) // s
        hi = ((i + 1) * m) // s
        assert np.all(pos >= lo) and np.all(pos < hi)
        assert np.array_equal(pos, F.sample_positions(n, m, seed=9).astype(np.int64))
        if m // s >= 2:  # strata of one position leave nothing to draw
            assert not np.array_equal(pos, F.sample_positions(n, m, seed=10).astype(np.int64))


def test_sample_size_is_one_percent_of_vertices():
    assert F.sample_count(10**6, 10**7) == 10000          # Section IV-C: 1% of |V|
    assert F.sample_count(1000, 10**6) == 4096             # floor for small graphs
    assert F.sample_count(10**6, 500) == 500               # never more samples than edges


def test_features_of_a_star():
    # every edge points at vertex 5: one destination, all coverage on it
    n, deg = 20000, 4
    O = np.arange(0, deg * n + 1, deg, dtype=np.int64)
    D = np.full(deg * n, 5, dtype=np.int32)
    f = F.features(O, D, False, seed=3)
    s = F.sample_count(n, D.size)
    assert np.allclose(f[4:8], 1.0) and np.allclose(f[8:11], 1.0)
    assert f[14] == 1.0                     # the one bin holds every edge
    assert np.isclose(f[15], 1.0 / s)
    assert f[3] == 0.0 and np.isclose(f[0], np.log2(n + 1) / 32)


def test_features_of_a_cycle_and_uniform():
    n = 50000
    O = np.arange(n + 1, dtype=np.int64)
    D = ((np.arange(n) + 1) % n).astype(np.int32)
    f = F.features(O, D, True, seed=3)
    s = F.sample_count(n, n)
    # each destination sampled at most once; distance 1 except the wrap
    assert f[4] == 0.0 and np.isclose(f[15], 1.0)
    assert f[12] >= (s - 1) / s and f[3] == 1.0
    rng = np.random.default_rng(0)
    O = np.arange(0, 16 * n + 1, 16, dtype=np.int64)
    D = rng.integers(0, n, size=16 * n).astype(np.int32)
    f = F.features(O, D, False, seed=3)
    assert f[14] == 0.0                     # no bin near 8K edges
    assert 0.2 < f[11] < 0.45               # mean |dst - src| / n of uniform pairs is 1/3


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(rng) + rng.normal(0, 0.05, M.NUM_PARAMS)
    x = rng.random((7, M.F))
    t = rng.normal(size=(7, M.G))
    g = M.gradient(p, x, t)
    idx = rng.choice(M.NUM_PARAMS, 300, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (M.loss(p + e, x, t) - M.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_mlp_forward_hand_example():
    # identity-like weights: y = relu(relu(x W1) W2) W3 with W picking coordinates
    p = np.zeros(M.NUM_PARAMS)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    W1[0, 0] = 2.0
    W1[1, 1] = -1.0
    W2[0, 0] = 1.0
    W2[1, 1] = 1.0
    W3[0, 3] = 1.5
    b3[:] = 0.25
    x = np.zeros((1, M.F))
    x[0, 0], x[0, 1] = 3.0, 4.0
    y, _ = M.forward(p, x)
    expect = np.full(M.G, 0.25)
    expect[3] += 1.5 * 6.0          # relu(2*3)=6 -> 6 -> *1.5; the -4 branch is cut by ReLU
    assert np.allclose(y[0], expect)


def test_adam_first_step_moves_by_lr():
    # with bias correction the first step is lr * g/|g| (eps aside)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, _, _ = M.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)


def mixed_frequency_graph():
    """A graph small enough (m <= 4096) that the sample is every edge once:
    s = m, so each stratum is one position.  Destinations, by construction:
      5 hubs 70000..70004, 40 in-edges each from sources 0..39   (bucket 5)
      10 vertices 1000..1009, 10 in-edges each from v+1..v+10     (bucket 3)
      1500 vertices 20000..21499, from v+200 and from v+60000     (bucket 1)
      500 vertices 90000..90499, one in-edge each from v-80000    (bucket 0)
    n = 100000, m = 200 + 100 + 3000 + 500 = 3800."""
    pairs = []
    for h in range(5):
        pairs += [(u, 70000 + h) for u in range(40)]
    for k in range(10):
        pairs += [(1000 + k + j, 1000 + k) for j in range(1, 11)]
    for k in range(1500):
        pairs += [(20000 + k + 200, 20000 + k), (20000 + k + 60000, 20000 + k)]
    for k in range(500):
        pairs += [(90000 + k - 80000, 90000 + k)]
    n = 100000
    pairs.sort(key=lambda p: p[0])  # stable: CSR order by source
    src = np.array([p[0] for p in pairs], dtype=np.int64)
    D = np.array([p[1] for p in pairs], dtype=np.int32)
    O = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int64)
    return O, D, src


def test_features_of_a_mixed_frequency_graph_by_hand():
    """Every feature computed by hand from the construction above, including
    the share of a partly taken frequency bucket in the coverage estimate."""
    O, D, src = mixed_frequency_graph()
    n, m = O.size - 1, D.size
    assert m == 3800 and F.sample_count(n, m) == m
    assert np.array_equal(F.sample_positions(n, m, seed=11).astype(np.int64), np.arange(m))
    f = F.features(O, D, True, seed=11).astype(np.float64)
    s = 3800.0
    assert np.isclose(f[0], np.log2(100001) / 32)
    assert np.isclose(f[1], np.log2(3801) / 40)                  # log m
    assert np.isclose(f[2], np.log2(3800 / 100000 + 1) / 8)      # edge factor
    assert f[3] == 1.0
    # edges into destinations sampled at least 2, 4, 16, 64 times
    assert np.isclose(f[4], (200 + 100 + 3000) / s)
    assert np.isclose(f[5], (200 + 100) / s)
    assert np.isclose(f[6], 200 / s)
    assert f[7] == 0.0
    # coverage of the 1024 most frequent: the 5 hubs (200), the 10 (100),
    # then 1009 of the 1500 twice-sampled vertices at 2 each (partial bucket)
    assert np.isclose(f[8], (200 + 100 + 1009 * 2) / s)
    assert np.isclose(f[9], 1.0) and np.isclose(f[10], 1.0)      # 2015 keys < 2^14
    dist_sum = (sum(70000 + h - u for h in range(5) for u in range(40)) + 10 * sum(range(1, 11))
                + 1500 * (200 + 60000) + 500 * 80000)
    assert np.isclose(f[11], dist_sum / (s * n), rtol=1e-6)
    assert np.isclose(f[12], (100 + 1500) / s)                   # |dst - src| < 256
    assert np.isclose(f[13], (100 + 1500 + 1500) / s)            # |dst - src| < 65536
    assert f[14] == 0.0                                           # no 256-vertex bin near 8K edges
    assert np.isclose(f[15], (5 + 10 + 1500 + 500) / s)          # distinct destinations

