"""Pins of the oracle against facts that do not come from the oracle itself.

Each pin is independent of the oracle's code: Python's stable sort, numpy's
stable argsort, scipy's CSR->CSC conversion, brute force over every tiny CSR,
closed forms (T[v] = #{e : D[e] < v}), the invariants the paper states
(transposing twice returns the input, Section II-A; the insertion points end
one slot further, Algorithm 1 footnote 1), special graphs with known
transposes, and the Fig. 1 prose of Section II-A.  A last group plants
mistakes in a copy of the oracle's output and checks that the pins catch them.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def stable_reference(O, D, P):
    """Definition by Python's stable sort of edge positions keyed by destination."""
    n = len(O) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(O)))
    order = sorted(range(len(D)), key=lambda e: int(D[e]))
    T = [0] * (n + 1)
    for v in range(n):
        T[v + 1] = T[v] + sum(1 for d in D if int(d) == v)
    S = [int(src[e]) for e in order]
    Q = [int(P[e]) for e in order] if P is not None else None
    return T, S, Q


def check_invariants(O, D, P, T, S, Q):
    """Properties any correct stable transposition has; returns a list of failures."""
    O, D = np.asarray(O), np.asarray(D)
    T, S = np.asarray(T), np.asarray(S)
    n, m = O.size - 1, D.size
    bad = []
    if T.size != n + 1 or T[0] != 0 or T[-1] != m:
        bad.append("T ends")
    if np.any(np.diff(T) < 0):
        bad.append("T monotone")
    # closed form of the offsets: T[v] = #{e : D[e] < v}
    if not np.array_equal(T, np.searchsorted(np.sort(D, kind="stable"), np.arange(n + 1), side="left")):
        bad.append("T closed form")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(O))
    # each list ascends by source
    dst_of_slot = np.repeat(np.arange(n, dtype=np.int64), np.diff(T))
    same = dst_of_slot[1:] == dst_of_slot[:-1]
    if np.any((np.diff(S.astype(np.int64)) < 0) & same):
        bad.append("lists ascend")
    # multiset of (src, dst, payload) preserved
    a = sorted(zip(src.tolist(), D.tolist(), (P.tolist() if P is not None else [0] * m)))
    b = sorted(zip(S.tolist(), dst_of_slot.tolist(), (list(Q) if Q is not None else [0] * m)))
    if a != b:
        bad.append("edge multiset")
    return bad


def test_fig1_prose_golden():
    vals = {}
    with open(os.path.join(GOLDEN, "fig1_prose.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            vals[k] = [int(x) for x in v]
    # a 4-vertex graph consistent with the prose: 0->{1,2}, 3->0 (+ 1->2, 2->3)
    O = np.array([0, 2, 3, 4, 5])
    D = np.array([1, 2, 2, 3, 0], dtype=np.int32)
    assert O[:2].tolist() == vals["csr_offsets_prefix"]
    assert D[:2].tolist() == vals["csr_edges_prefix"]
    T, S, _ = oracle.transpose(O, D)
    assert T[:2].tolist() == vals["csc_offsets_prefix"]
    assert S[:1].tolist() == vals["csc_edges_prefix"]


def all_tiny_csrs(max_n=3, max_m=4):
    """Every CSR with n <= max_n and m <= max_m (any list order, duplicates, self-loops)."""
    for n in range(0, max_n + 1):
        for m in range(0, max_m + 1 if n > 0 else 1):
            for dsts in itertools.product(range(n), repeat=m):
                # every way to cut the m edges into n consecutive lists
                for cuts in itertools.combinations_with_replacement(range(m + 1), max(n - 1, 0)):
                    O = [0] + list(cuts) + [m] if n > 0 else [0]
                    yield np.array(O, dtype=np.int64), np.array(dsts, dtype=np.int32)


def test_bruteforce_all_tiny_graphs():
    count = 0
    for O, D in all_tiny_csrs():
        P = np.arange(D.size, dtype=np.uint32) + 7  # payload = position tag
        T, S, Q = oracle.transpose(O, D, P)
        rT, rS, rQ = stable_reference(O, D, P)
        assert T.tolist() == rT and S.tolist() == rS and Q.tolist() == rQ, (O, D)
        pT, pS, pQ = oracle.transpose_py(O, D, P)
        assert pT == rT and pS == rS and pQ == rQ
        count += 1
    assert count == 1684  # every CSR with n <= 3 vertices and m <= 4 edges


@pytest.mark.parametrize("seed", range(6))
def test_random_vs_numpy_and_scipy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    deg = rng.integers(0, 12, size=n)
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    m = int(O[-1])
    # skewed destinations with many duplicates, unsorted lists
    D = (rng.zipf(1.6, size=m) % n).astype(np.int32)
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    T, S, Q = oracle.transpose(O, D, P)
    order = np.argsort(D, kind="stable")
    src = np.repeat(np.arange(n), deg)
    assert np.array_equal(S, src[order])
    assert np.array_equal(Q, P[order])
    assert np.array_equal(T, np.concatenate([[0], np.cumsum(np.bincount(D, minlength=n))]))
    # scipy: carry the edge position + 1 as the value so the order is visible
    A = sp.csr_matrix((np.arange(1, m + 1, dtype=np.int64), D, O), shape=(n, n))
    C = A.tocsc()
    assert np.array_equal(C.indptr, T)
    assert np.array_equal(C.indices, S)
    assert np.array_equal(C.data - 1, order)
    assert check_invariants(O, D, P, T, S, Q) == []


def test_transpose_twice_is_identity():
    # Section II-A: the transposed of a transposed format equals the original
    # (with ascending lists the CSR is the unique stable form)
    rng = np.random.default_rng(11)
    n = 300
    deg = rng.integers(0, 20, size=n)
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    D = np.concatenate([np.sort(rng.integers(0, n, size=d)) for d in deg]).astype(np.int32)
    P = rng.integers(0, 2**32, size=D.size, dtype=np.uint64).astype(np.uint32)
    T, S, Q = oracle.transpose(O, D, P)
    O2, D2, P2 = oracle.transpose(T, S, Q)
    assert np.array_equal(O2, O) and np.array_equal(D2, D) and np.array_equal(P2, P)


def test_symmetric_graph_csc_equals_csr():
    # Section II-A: for undirected graphs CSR and CSC coincide
    rng = np.random.default_rng(5)
    n = 200
    E = set()
    for _ in range(900):
        u, v = map(int, rng.integers(0, n, size=2))
        E.add((u, v)); E.add((v, u))
    E = sorted(E)
    D = np.array([v for _, v in E], dtype=np.int32)
    O = np.searchsorted(np.array([u for u, _ in E]), np.arange(n + 1)).astype(np.int64)
    T, S, _ = oracle.transpose(O, D)
    assert np.array_equal(T, O) and np.array_equal(S, D)


def test_special_graphs():
    n = 17
    # all self-loops, two per vertex
    O = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    D = np.repeat(np.arange(n), 2).astype(np.int32)
    T, S, _ = oracle.transpose(O, D)
    assert np.array_equal(T, O) and np.array_equal(S, D)
    # star into vertex 0: every vertex points at 0 three times
    O = np.arange(0, 3 * n + 1, 3, dtype=np.int64)
    D = np.zeros(3 * n, dtype=np.int32)
    T, S, _ = oracle.transpose(O, D)
    assert T.tolist() == [0] + [3 * n] * n
    assert S.tolist() == np.repeat(np.arange(n), 3).tolist()
    # directed cycle u -> u+1 mod n
    O = np.arange(n + 1, dtype=np.int64)
    D = ((np.arange(n) + 1) % n).astype(np.int32)
    T, S, _ = oracle.transpose(O, D)
    assert T.tolist() == list(range(n + 1))
    assert S.tolist() == [(v - 1) % n for v in range(n)]


def test_empty_cases():
    T, S, Q = oracle.transpose(np.array([0]), np.array([], dtype=np.int32), np.array([], dtype=np.uint32))
    assert T.tolist() == [0] and S.size == 0 and Q.size == 0
    T, S, _ = oracle.transpose(np.zeros(6, dtype=np.int64), np.array([], dtype=np.int32))
    assert T.tolist() == [0] * 6 and S.size == 0


def test_invalid_graphs_rejected():
    good_O, good_D = np.array([0, 1, 2]), np.array([1, 0], dtype=np.int32)
    assert oracle.validate(good_O, good_D) == oracle.ORC_OK
    assert oracle.validate(np.array([0, 2, 1]), good_D) == oracle.ORC_EGRAPH   # decreasing
    assert oracle.validate(np.array([1, 1, 2]), good_D) == oracle.ORC_EGRAPH   # O[0] != 0
    assert oracle.validate(np.array([0, 1, 1]), good_D) == oracle.ORC_EGRAPH   # O[n] != m
    assert oracle.validate(good_O, np.array([2, 0], dtype=np.int32)) == oracle.ORC_EGRAPH
    assert oracle.validate(good_O, np.array([-1, 0], dtype=np.int32)) == oracle.ORC_EGRAPH
    with pytest.raises(oracle.OracleError):
        oracle.transpose(np.array([0, 2, 1]), good_D)


def test_payload_bits_travel_exactly():
    # NaN, -0.0, denormals and infinities are moved as words, never as floats
    words = np.array([0x7FC00001, 0x80000000, 0x00000001, 0x7F800000, 0xFF800000, 0x3F800000],
                     dtype=np.uint32)
    O = np.array([0, 3, 6], dtype=np.int64)
    D = np.array([1, 0, 1, 1, 0, 0], dtype=np.int32)
    T, S, Q = oracle.transpose(O, D, words)
    assert Q.tolist() == [words[1], words[4], words[5], words[0], words[2], words[3]]
    assert S.tolist() == [0, 1, 1, 0, 0, 1]


def test_slice_matches_full():
    rng = np.random.default_rng(3)
    n = 1000
    deg = rng.integers(0, 30, size=n)
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    D = (rng.zipf(1.4, size=int(O[-1])) % n).astype(np.int32)
    P = np.arange(D.size, dtype=np.uint32)
    T, S, Q = oracle.transpose(O, D, P)
    for lo, hi in [(0, 1), (0, n), (5, 17), (400, 1000), (999, 1000), (300, 300)]:
        Ts, Ss, Qs = oracle.transpose_slice(O, D, P, lo, hi)
        assert np.array_equal(Ts, T[lo:hi + 1])
        assert np.array_equal(Ss, S[T[lo]:T[hi]]) and np.array_equal(Qs, Q[T[lo]:T[hi]])


def test_generated_workload_invariants():
    import gen
    O, D, P = gen.rmat(12, 16, seed=1, permute=True, payload=True)
    T, S, Q = oracle.transpose(O, D, P)
    assert check_invariants(O, D, P, T, S, Q) == []
    order = np.argsort(D, kind="stable")
    assert np.array_equal(Q, P[order])


# ---- planted mistakes: each must be caught by at least one pin ----------------------

def _planted_outputs():
    rng = np.random.default_rng(8)
    n = 60
    deg = rng.integers(1, 9, size=n)
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    D = (rng.zipf(1.5, size=int(O[-1])) % n).astype(np.int32)
    D[:3] = 0  # guarantee a duplicate run (0 -> 0 three times)
    P = np.arange(D.size, dtype=np.uint32)
    T, S, Q = oracle.transpose(O, D, P)
    return O, D, P, T, S, Q


@pytest.mark.parametrize("mistake", ["swap_in_list", "offset_shift", "drop_edge", "transpose_operand",
                                     "tie_order", "wrong_source"])
def test_pins_catch_planted_mistakes(mistake):
    O, D, P, T, S, Q = _planted_outputs()
    T, S, Q = T.copy(), S.copy(), Q.copy()
    if mistake == "swap_in_list":
        v = int(np.argmax(np.diff(T)))
        a = int(T[v])
        S[a], S[a + 1] = S[a + 1], S[a]
        Q[a], Q[a + 1] = Q[a + 1], Q[a]
        if S[a] == S[a + 1]:
            S[a] += 1
    elif mistake == "offset_shift":
        T[5] += 1
    elif mistake == "drop_edge":
        S, Q = S[:-1], Q[:-1]
        T[-1] -= 1
    elif mistake == "transpose_operand":
        S = D.copy()
    elif mistake == "tie_order":
        # the three 0 -> 0 edges: swap their payloads (ties must follow CSR order)
        Q[0], Q[1] = Q[1], Q[0]
    elif mistake == "wrong_source":
        S[3] = (S[3] + 1) % (O.size - 1)
    order = np.argsort(D, kind="stable")
    src = np.repeat(np.arange(O.size - 1), np.diff(O))
    try:
        inv_bad = bool(check_invariants(O, D, P, T, S, Q))
    except ValueError:  # shape mismatch is a failure too
        inv_bad = True
    caught = inv_bad or not (
        np.array_equal(S, src[order]) and np.array_equal(Q, P[order]))
    assert caught
