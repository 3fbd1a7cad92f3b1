"""GPU: the paper's own methods (HLH / PoTra and Atomic GT) against the oracle.

Both leave the order inside a CSC list to the atomics, as the paper does, so
the check is: offsets bit-exact, and every list equal to the oracle's list as
a multiset of (source, payload) pairs.  Every case prints its name first.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from test_gpu_parity import random_csr, to_dev

pytestmark = pytest.mark.gpu

STRATEGIES = {"hlh": 1, "atomic": 2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def canonical(T, S, Q):
    """Each list sorted by (source, payload): the unique representative of
    the multiset."""
    n = T.size - 1
    vid = np.repeat(np.arange(n), np.diff(T))
    keys = (S,) if Q is None else (Q, S)
    order = np.lexsort(keys + (vid,))
    return S[order], (Q[order] if Q is not None else None)


def assert_unordered_parity(O, D, P, dev, label, strategy, **opt):
    import paper_2501_06872_amd as gt
    say(f"[case] {label} strategy={strategy} n={len(O) - 1} m={len(D)} payload={P is not None} opt={opt}")
    g = to_dev(O, D, P, dev)
    plan = gt.Plan([g], gt.make_options(strategy=STRATEGIES[strategy], **opt))
    T, S, Q = plan.run(*g)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    T, S = T.cpu().numpy(), S.cpu().numpy()
    Q = Q.cpu().numpy().view(np.uint32) if Q is not None else None
    rT, rS, rQ = oracle.transpose(O, D, P)
    assert np.array_equal(T, rT), f"{label}: offsets differ"
    cS, cQ = canonical(T, S, Q)
    oS, oQ = canonical(rT, rS, rQ)
    assert np.array_equal(cS, oS), f"{label}: list contents differ"
    if P is not None:
        assert np.array_equal(cQ, oQ), f"{label}: payloads differ"


@pytest.mark.parametrize("strategy", ["hlh", "atomic"])
def test_rmat_natural_and_permuted(hip_device, strategy):
    O, D, P = gen.workload("rmat16")
    assert_unordered_parity(O, D, P, hip_device, "rmat16", strategy)
    O, D, P = gen.rmat(18, 16, seed=2, permute=True, payload=True)
    assert_unordered_parity(O, D, P, hip_device, "rmat18p payload", strategy)


@pytest.mark.parametrize("strategy", ["hlh", "atomic"])
def test_hub_and_locality(hip_device, strategy):
    n = 50000  # every vertex points at vertex 7 three times: one hub
    O = np.arange(0, 3 * n + 1, 3, dtype=np.int64)
    D = np.full(3 * n, 7, dtype=np.int32)
    P = np.arange(3 * n, dtype=np.uint32)
    assert_unordered_parity(O, D, P, hip_device, "star", strategy)
    O, D, P = gen.geometric(1 << 17, 8, seed=5, p=0.01, payload=True)
    assert_unordered_parity(O, D, P, hip_device, "geometric", strategy)
    O, D, P = gen.uniform((1 << 16) + 77, 4, seed=6)
    assert_unordered_parity(O, D, P, hip_device, "uniform ragged n", strategy)


@pytest.mark.parametrize("strategy", ["hlh", "atomic"])
def test_unsorted_duplicates_and_degenerate(hip_device, strategy):
    rng = np.random.default_rng(44)
    O, D, P = random_csr(rng, 30000, 9, skew=1.3, sorted_lists=False, payload=True)
    assert_unordered_parity(O, D, P, hip_device, "zipf unsorted", strategy)
    e32 = np.array([], dtype=np.int32)
    assert_unordered_parity(np.array([0]), e32, None, hip_device, "n=0", strategy)
    assert_unordered_parity(np.zeros(6, dtype=np.int64), e32, None, hip_device, "m=0", strategy)
    n = 70001  # self-loops and a cycle
    O = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    D = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).ravel().astype(np.int32)
    assert_unordered_parity(O, D, None, hip_device, "self-loops + cycle", strategy)
    n = 300000  # one source with 100k out-edges crossing several chunks
    deg = np.zeros(n, dtype=np.int64)
    deg[3] = 100000
    deg[10:5000] = 3
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    D = rng.integers(0, n, size=int(O[-1])).astype(np.int32)
    assert_unordered_parity(O, D, None, hip_device, "long list", strategy)


def test_hlh_small_table(hip_device):
    O, D, P = gen.rmat(17, 16, seed=9, permute=False, payload=True)
    for k in (1, 16, 300):
        assert_unordered_parity(O, D, P, hip_device, f"rmat17 hdv_max={k}", "hlh", hdv_max=k)


def test_probe_picks_a_method_and_stays_exact(hip_device):
    # the probe of Section IV-C: HLH or Atomic GT, whichever counts faster on
    # a sixteenth of the chunks; either way the result is the transposition
    import paper_2501_06872_amd as gt
    cases = [("star", None), ("rmat18", gen.rmat(18, 16, seed=3, permute=False, payload=True)),
             ("uniform", gen.uniform(1 << 18, 8, seed=4))]
    n = 80000
    star = (np.arange(0, 4 * n + 1, 4, dtype=np.int64), np.full(4 * n, 11, dtype=np.int32), None)
    cases[0] = ("star", star)
    for label, (O, D, P) in cases:
        say(f"[case] probe {label}")
        g = to_dev(O, D, P, hip_device)
        plan = gt.Plan([g], gt.make_options(strategy=gt.STRATEGY_PROBE))
        picked = plan.strategy()
        say(f"  probe kept {'HLH' if picked == gt.STRATEGY_HLH else 'Atomic GT'}")
        assert picked in (gt.STRATEGY_HLH, gt.STRATEGY_ATOMIC)
        T, S, Q = plan.run(*g)
        torch.cuda.synchronize()
        rT, rS, rQ = oracle.transpose(O, D, P)
        T, S = T.cpu().numpy(), S.cpu().numpy()
        Q = Q.cpu().numpy().view(np.uint32) if Q is not None else None
        assert np.array_equal(T, rT)
        cS, cQ = canonical(T, S, Q)
        oS, oQ = canonical(rT, rS, rQ)
        assert np.array_equal(cS, oS)
        if P is not None:
            assert np.array_equal(cQ, oQ)


@pytest.mark.parametrize("mode", ["static", "steal"])
@pytest.mark.parametrize("strategy", ["hlh", "atomic"])
def test_step3_static_and_two_phase(hip_device, strategy, mode):
    """Step 3 with one chunk per resident workgroup (static), and in the two
    phases of Section V-F (each workgroup scatters the head of its chunk,
    then claims tail parts atomically): offsets exact and every list equal to
    the oracle's as a multiset, on skewed, hub, tiny and ragged inputs, with
    the per-chunk time stamps recorded."""
    import paper_2501_06872_amd as gt
    flags = (gt.FLAG_STEP3_STEAL if mode == "steal" else gt.FLAG_STEP3_STATIC) | gt.FLAG_STEP3_TIMES
    O, D, P = gen.rmat(19, 16, seed=12, permute=False, payload=True)
    assert_unordered_parity(O, D, P, hip_device, f"rmat19 {mode}", strategy, flags=flags)
    n = 60000  # a hub: every vertex points at vertex 5 four times
    O = np.arange(0, 4 * n + 1, 4, dtype=np.int64)
    D = np.full(4 * n, 5, dtype=np.int32)
    assert_unordered_parity(O, D, np.arange(4 * n, dtype=np.uint32), hip_device, f"star {mode}", strategy,
                            flags=flags)
    # fewer edges than chunks, and a ragged count
    rng = np.random.default_rng(8)
    O, D, P = random_csr(rng, 700, 3, payload=True)
    assert_unordered_parity(O, D, P, hip_device, f"tiny {mode}", strategy, flags=flags)
    O, D, _ = gen.uniform((1 << 17) + 333, 7, seed=2)
    assert_unordered_parity(O, D, None, hip_device, f"uniform ragged {mode}", strategy, flags=flags)


def test_step3_time_stamps(hip_device):
    import paper_2501_06872_amd as gt
    from paper_2501_06872_amd import step3
    O, D, P = gen.rmat(18, 16, seed=4, permute=True)
    g = to_dev(O, D, P, hip_device)
    for mode, flag in (("static", gt.FLAG_STEP3_STATIC), ("steal", gt.FLAG_STEP3_STEAL)):
        say(f"[case] step-3 time stamps, {mode}")
        plan = gt.Plan([g], gt.make_options(strategy=gt.STRATEGY_HLH, flags=flag | gt.FLAG_STEP3_TIMES))
        plan.run(*g)
        torch.cuda.synchronize()
        st = plan.step3_times()
        assert st.shape[1] == 3 and st.shape[0] >= 1
        assert np.all(st[:, 0] <= st[:, 1]) and np.all(st[:, 1] <= st[:, 2])
        bal = step3.balance(st, plan.step3_clock_hz())
        say(f"  {st.shape[0]} chunks, imbalance {bal['imbalance']:.3f}")
        assert 0.0 <= bal["imbalance"] < 1.0


def test_hlh_sixteen_bit_counters_carry(hip_device):
    """Step 1's HDV counters are 16-bit with a carry into the part's high
    counter (Algorithm 2): a hub whose edges fill whole chunks wraps its low
    counter exactly once per chunk (2^20 edges: 16 chunks of 65536) and twice
    per chunk when chunks hold 2^17 edges (2^25 edges in the static
    chunking: one chunk per resident workgroup).  The offsets stay exact and
    every list equals the oracle's as a multiset."""
    import paper_2501_06872_amd as gt
    for m, flags in ((1 << 20, 0), (1 << 25, gt.FLAG_STEP3_STATIC)):
        n = 1 << 20
        O = np.arange(0, m + 1, m // n, dtype=np.int64)
        D = np.full(m, 12345, dtype=np.int32)
        D[::1001] = np.arange(D[::1001].size, dtype=np.int32) % n  # a few other destinations
        for u in range(0, n, max(1, n // 4096)):
            D[O[u]:O[u + 1]].sort()
        if m == 1 << 20:
            P = np.arange(m, dtype=np.uint32)
        else:
            P = None
        # lists must ascend for the generator's reading, not for the method
        assert_unordered_parity(O, D, P, hip_device, f"hub m=2^{m.bit_length() - 1}", "hlh", flags=flags)
