"""Checks of the seeded input generators (CPU only)."""
import numpy as np

import gen


def test_rmat_first_level_quadrants():
    # fraction of edges whose top (src bit, dst bit) falls in each quadrant ~ (a, b, c, d)
    s = 14
    O, D, _ = gen.rmat(s, 16, seed=1)
    src = np.repeat(np.arange(1 << s), np.diff(O))
    sb, db = src >> (s - 1), D.astype(np.int64) >> (s - 1)
    m = D.size
    freq = [np.count_nonzero((sb == i) & (db == j)) / m for i, j in ((0, 0), (0, 1), (1, 0), (1, 1))]
    for f, p in zip(freq, gen.RMAT_G500):
        assert abs(f - p) < 0.01, (freq, gen.RMAT_G500)


def test_rmat_exact_edge_count_and_sorted_lists():
    O, D, P = gen.rmat(12, 16, seed=9, permute=True, payload=True)
    assert O[0] == 0 and O[-1] == 16 << 12 and np.all(np.diff(O) >= 0)
    assert D.min() >= 0 and D.max() < 1 << 12
    for u in range(0, 1 << 12, 97):
        lst = D[O[u]:O[u + 1]]
        assert np.all(np.diff(lst) >= 0)
    f = P.view(np.float32)
    assert np.all((f >= 0) & (f < 1))


def test_non_power_of_two_rmat():
    n = 3000
    O, D, _ = gen.generate(gen.FAM_RMAT, n, 8, seed=4)
    assert O.size == n + 1 and O[-1] == 8 * n and D.max() < n


def test_uniform_and_geometric_shapes():
    n = 1 << 16
    O, D, _ = gen.uniform(n, 16, seed=3)
    assert np.all(np.diff(O) == 16)
    indeg = np.bincount(D, minlength=n)
    assert abs(indeg.mean() - 16) < 1e-9 and abs(indeg.var() - 16) < 1.0
    O, D, _ = gen.geometric(n, 16, seed=3, p=0.01)
    src = np.repeat(np.arange(n), 16)
    off = (D.astype(np.int64) - src) % n
    assert off.min() >= 1 and abs(off.mean() - 100) < 2.0   # mean of Geometric(0.01) on {1, 2, ...}


def test_permutation_is_bijection():
    for n in (1, 2, 1000, 1 << 16, 12345):
        ids = np.arange(n, dtype=np.int32)
        p = gen.permutation(n, 77, ids)
        assert np.array_equal(np.sort(p), ids)
        assert np.array_equal(gen.permutation(n, 77, p, inverse=True), ids)


def test_determinism():
    a = gen.rmat(13, 8, seed=5, permute=True, payload=True)
    b = gen.rmat(13, 8, seed=5, permute=True, payload=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c = gen.rmat(13, 8, seed=6, permute=True, payload=True)
    assert not np.array_equal(a[1], c[1])


def test_batch_specs_shape():
    specs = gen.batch_specs(512)
    assert len(specs) == 512
    assert sum(s["payload"] for s in specs) == 256
    ns = np.array([s["n"] for s in specs])
    assert ns.min() >= 1 << 10 and ns.max() < 1 << 22
    assert {s["ef"] for s in specs} == {4, 8, 16, 32}
    assert {s["family"] for s in specs} == {0, 1, 2}
