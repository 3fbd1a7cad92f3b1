"""GPU parity: the HIP transposition against the CPU oracle, bit for bit.

Inputs are seeded and synthetic.  Every case prints its name before it runs.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(O, D, P, dev):
    O_t = torch.from_numpy(np.ascontiguousarray(O)).to(dev)
    D_t = torch.from_numpy(np.ascontiguousarray(D)).to(dev)
    P_t = torch.from_numpy(np.ascontiguousarray(P).view(np.int32)).to(dev) if P is not None else None
    return O_t, D_t, P_t


def gpu_transpose(O, D, P, dev, **opt):
    import paper_2501_06872_amd as gt
    O_t, D_t, P_t = to_dev(O, D, P, dev)
    options = gt.make_options(**opt) if opt else None
    plan = gt.Plan([(O_t, D_t, P_t)], options)
    T, S, Q = plan.run(O_t, D_t, P_t)
    torch.cuda.synchronize()
    st = plan.device_status()
    params = plan.params()
    params["packed"] = plan.packed()
    return (T.cpu().numpy(), S.cpu().numpy(), Q.cpu().numpy().view(np.uint32) if Q is not None else None,
            st, params)


def assert_parity(O, D, P, dev, label, **opt):
    say(f"[case] {label} n={len(O) - 1} m={len(D)} payload={P is not None} opt={opt}")
    T, S, Q, st, params = gpu_transpose(O, D, P, dev, **opt)
    assert st == 0, f"device status {st}"
    rT, rS, rQ = oracle.transpose(O, D, P)
    assert np.array_equal(T, rT), f"{label}: offsets differ"
    assert np.array_equal(S, rS), f"{label}: sources differ at {np.flatnonzero(S != rS)[:5]}"
    if P is not None:
        assert np.array_equal(Q, rQ), f"{label}: payload differs"
    return params


def random_csr(rng, n, avg_deg, skew=None, sorted_lists=True, payload=False):
    deg = rng.poisson(avg_deg, size=n)
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    m = int(O[-1])
    if skew:
        D = (rng.zipf(skew, size=m) - 1) % max(n, 1)
    else:
        D = rng.integers(0, max(n, 1), size=m)
    D = D.astype(np.int32)
    if sorted_lists:
        for u in range(n):
            D[O[u]:O[u + 1]].sort()
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32) if payload else None
    return O, D, P


def test_rmat16_default(hip_device):
    O, D, P = gen.workload("rmat16")
    params = assert_parity(O, D, P, hip_device, "rmat16 (R-MAT scale 16, ef 16, seed 1)")
    say("params", params)


@pytest.mark.parametrize("payload", [False, True])
def test_rmat_permuted_small(hip_device, payload):
    O, D, P = gen.rmat(18, 16, seed=2, permute=True, payload=payload)
    assert_parity(O, D, P, hip_device, "rmat18 permuted")


def test_empty_and_degenerate(hip_device):
    e32 = np.array([], dtype=np.int32)
    assert_parity(np.array([0]), e32, None, hip_device, "n=0")
    assert_parity(np.array([0, 0]), e32, None, hip_device, "n=1 m=0")
    assert_parity(np.zeros(1001, dtype=np.int64), e32, None, hip_device, "n=1000 m=0")
    assert_parity(np.array([0, 5]), np.zeros(5, dtype=np.int32), np.arange(5, dtype=np.uint32), hip_device,
                  "n=1 five self-loops")
    assert_parity(np.array([0, 1, 1]), np.array([1], dtype=np.int32), None, hip_device, "n=2 one edge")


def test_star_into_one_vertex(hip_device):
    # every vertex points at vertex 7 (in-degree = m: the multi-tile bin path)
    n = 50000
    O = np.arange(0, 3 * n + 1, 3, dtype=np.int64)
    D = np.full(3 * n, 7, dtype=np.int32)
    P = np.arange(3 * n, dtype=np.uint32)
    assert_parity(O, D, P, hip_device, "star into vertex 7")


def test_self_loops_and_cycle(hip_device):
    n = 70001
    O = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    D = np.repeat(np.arange(n), 2).astype(np.int32)
    assert_parity(O, D, None, hip_device, "all self-loops")
    O = np.arange(n + 1, dtype=np.int64)
    D = ((np.arange(n) + 1) % n).astype(np.int32)
    assert_parity(O, D, None, hip_device, "directed cycle")


def test_unsorted_lists_duplicates_payload_bits(hip_device):
    rng = np.random.default_rng(21)
    O, D, P = random_csr(rng, 20000, 9, skew=1.3, sorted_lists=False, payload=True)
    special = np.array([0x7FC00001, 0x80000000, 0x00000001, 0x7F800000, 0xFF800000], dtype=np.uint32)
    P[: special.size * 50] = np.tile(special, 50)
    assert_parity(O, D, P, hip_device, "unsorted lists, duplicates, NaN/-0/denormal payload")


def test_one_source_spanning_many_tiles(hip_device):
    # vertex 3 has 100k out-edges: its list crosses several 8K tiles; many empty rows
    n = 300000
    deg = np.zeros(n, dtype=np.int64)
    deg[3] = 100000
    deg[n - 1] = 17
    deg[1000:1100] = 5
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    rng = np.random.default_rng(3)
    D = np.sort(rng.integers(0, n, size=int(O[-1]))).astype(np.int32)
    D[: 40000] = 12345  # a duplicate run crossing tile boundaries
    D[:100000].sort()
    assert_parity(O, D, None, hip_device, "one source spanning tiles")


@pytest.mark.parametrize("n,avg,skew,payload", [
    (3, 2, None, False), (1000, 5, 1.5, True), (4097, 16, None, False), (65539, 16, 1.2, True),
    (300001, 7, 1.4, False), (1 << 20, 3, None, True),
])
def test_random_graphs_default_params(hip_device, n, avg, skew, payload):
    rng = np.random.default_rng(n)
    O, D, P = random_csr(rng, n, avg, skew=skew, payload=payload)
    assert_parity(O, D, P, hip_device, f"random n={n} avg={avg} skew={skew}")


def test_bins_of_many_chunks(hip_device):
    # one bin of ~88 work items (the wider column-prefix launch for bins of
    # more than 64 chunks), one of ~30 and many small ones
    rng = np.random.default_rng(21)
    n, m = 20_000, 1_200_000
    src = np.sort(rng.integers(0, n, size=m))
    D = rng.integers(0, n, size=m).astype(np.int32)
    u = rng.random(m)
    D[u < 0.6] = 3
    hit = (u >= 0.6) & (u < 0.8)
    D[hit] = rng.integers(512, 1024, size=int(hit.sum()))
    order = np.lexsort((D, src))
    src, D = src[order], D[order]
    O = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int64)
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    assert_parity(O, D, P, hip_device, "bins of many chunks", policy=1, fine_bits=9, digit_bits=8, variant=1)


@pytest.mark.parametrize("share", [1.0, 0.9, 0.3])
def test_hub_rows(hip_device, share):
    # one destination takes `share` of a bin spanning many work items: rows of
    # the bin are wholly, mostly or partly that destination (the single-key
    # row paths of the chunk counts and of the placement ranking)
    rng = np.random.default_rng(int(share * 100))
    n, m = 4096, 70_000
    src = np.sort(rng.integers(0, n, size=m))
    D = rng.integers(0, 512, size=m).astype(np.int32)
    D[rng.random(m) < share] = 5
    D[: 1000] = rng.integers(512, n, size=1000)
    order = np.lexsort((D, src))
    src, D = src[order], D[order]
    O = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int64)
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    assert_parity(O, D, P, hip_device, f"hub rows {share}", policy=1, fine_bits=9, digit_bits=8, variant=1)
    assert_parity(O, D, None, hip_device, f"hub rows {share}, no payload")


@pytest.mark.parametrize("payload", [False, True])
def test_two_pass_intermediate_wide_ids(hip_device, payload):
    # 26-bit vertex IDs, 9 fine bits, digits of 8 and 9 bits: the key of the
    # intermediate between the passes cannot hold all fine bits, so the top
    # ones travel in the source word; a hub and a dense block make the
    # first-pass digits uneven
    rng = np.random.default_rng(5)
    n = (1 << 25) + 3
    m = 3_000_000
    src = np.sort(rng.integers(0, n, size=m))
    D = rng.integers(0, n, size=m).astype(np.int32)
    D[: m // 5] = n - 1
    D[m // 5: m // 3] = rng.integers(0, 1 << 12, size=m // 3 - m // 5)
    rng.shuffle(D)
    order = np.lexsort((D, src))
    src, D = src[order], D[order]
    O = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int64)
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32) if payload else None
    params = assert_parity(O, D, P, hip_device, "26-bit ids, two passes", policy=1, fine_bits=9, digit_bits=9,
                           variant=1)
    assert params["passes"] == 2 and params["packed"], params


def test_two_pass_intermediate_one_tile(hip_device):
    # every digit boundary of the first pass falls inside the only tile
    rng = np.random.default_rng(8)
    O, D, P = random_csr(rng, 5000, 1.2, payload=True)
    for fine_bits, digit_bits, packed in ((1, 6, True), (4, 4, False), (2, 7, True)):  # three passes: not packed
        params = assert_parity(O, D, P, hip_device, "one tile, two passes", policy=1, fine_bits=fine_bits,
                               digit_bits=digit_bits, variant=1)
        assert params["packed"] == packed, params


@pytest.mark.parametrize("payload", [False, True])
def test_sparse_sources_many_per_tile(hip_device, payload):
    # a dense head, then a long stretch of sources with zero or one edge: a
    # partition tile of the first pass spans up to ~10^5 sources there
    rng = np.random.default_rng(31)
    n = 400_000
    deg = np.zeros(n, dtype=np.int64)
    deg[:2000] = rng.integers(0, 40, size=2000)
    tail = rng.random(n - 2000) < 0.05
    deg[2000:][tail] = 1
    deg[-1] = 3
    O = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    m = int(O[-1])
    D = rng.integers(0, n, size=m).astype(np.int32)
    for u in np.flatnonzero(deg > 1):
        D[O[u]:O[u + 1]].sort()
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32) if payload else None
    assert_parity(O, D, P, hip_device, "sparse sources")
    assert_parity(O, D, P, hip_device, "sparse sources, 3 passes", policy=1, fine_bits=4, digit_bits=5, variant=1)


@pytest.mark.parametrize("payload", [False, True])
def test_bin_sizes_around_the_final_item(hip_device, payload):
    # 16 bins of 512 destinations (fine_bits 9) whose edge counts straddle
    # the k_final work item (empty, one row, partial rows, small bins spread
    # over the waves, just below / at / above one and two items), with a hub
    # inside some bins
    rng = np.random.default_rng(77)
    sizes = [0, 1, 63, 64, 65, 500, 4097, 8191, 8192, 8193, 9215, 9216, 9217, 18432, 18433, 30000]
    n = 512 * 64  # 48 more bins, empty: six coarse bits
    src, dst = [], []
    for b, sz in enumerate(sizes):
        d = rng.integers(0, 512, size=sz)
        if b % 3 == 0:
            d[: sz // 4] = 7  # a heavy destination
        dst.append(b * 512 + d)
        src.append(rng.integers(0, n, size=sz))
    src = np.concatenate(src).astype(np.int64)
    dst = np.concatenate(dst).astype(np.int32)
    order = np.lexsort((dst, src))
    src, D = src[order], dst[order]
    O = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))]).astype(np.int64)
    P = rng.integers(0, 2**32, size=D.size, dtype=np.uint64).astype(np.uint32) if payload else None
    for digit_bits in (4, 8):  # two passes, one pass
        assert_parity(O, D, P, hip_device, "bins around the item size", policy=1, fine_bits=9,
                      digit_bits=digit_bits, variant=1)


@pytest.mark.parametrize("fine_bits,digit_bits,variant", [
    (1, 4, 1), (4, 6, 3), (8, 10, 2), (9, 4, 1), (5, 10, 3), (7, 8, 2), (9, 10, 1), (6, 5, 1), (8, 9, 4), (3, 6, 4),
    (7, 10, 4), (7, 10, 2),  # one 10-bit pass: the 16-wave variants run the 8-wave tile
])
def test_parameter_sweep_same_output(hip_device, fine_bits, digit_bits, variant):
    # 1, 2 and 3 partition passes, every tile variant, narrow and wide bins
    O, D, P = gen.rmat(17, 8, seed=9, permute=True, payload=True)
    params = assert_parity(O, D, P, hip_device, "rmat17p sweep", policy=1, fine_bits=fine_bits,
                           digit_bits=digit_bits, variant=variant)
    say("params", params)


@pytest.mark.parametrize("flags", [0, 1])
def test_ten_bit_first_pass_without_payload(hip_device, flags):
    # 1024 digits with 512 threads: the tile-local digit scan reads entries
    # that other waves write (needs the barrier before it); one 10-bit pass,
    # then a 10-bit first pass of two, 32- and 64-bit look-back words
    O, D, P = gen.rmat(17, 16, seed=13, permute=False)
    assert_parity(O, D, P, hip_device, "rmat17 one 10-bit pass", policy=1, fine_bits=7, digit_bits=10, variant=1,
                  flags=flags)
    O, D, P = gen.uniform(1 << 20, 4, seed=14)
    assert_parity(O, D, P, hip_device, "uniform20 10+9-bit passes", policy=1, fine_bits=1, digit_bits=10, variant=1,
                  flags=flags)
    O, D, P = gen.rmat(19, 8, seed=15, permute=False, payload=True)
    assert_parity(O, D, P, hip_device, "rmat19 payload 10-bit", policy=1, fine_bits=9, digit_bits=10, variant=3,
                  flags=flags)


@pytest.mark.parametrize("payload", [False, True])
def test_wide_lookback_words(hip_device, payload):
    # the 64-bit look-back words of graphs with m >= 2^31, forced on a small graph
    O, D, P = gen.rmat(17, 8, seed=12, permute=True, payload=payload)
    assert_parity(O, D, P, hip_device, "rmat17p wide status", flags=1)


def test_determinism_repeated_runs(hip_device):
    import paper_2501_06872_amd as gt
    O, D, P = gen.rmat(19, 16, seed=4, permute=True, payload=True)
    say(f"[case] determinism rmat19p m={len(D)}")
    O_t, D_t, P_t = to_dev(O, D, P, hip_device)
    plan = gt.Plan([(O_t, D_t, P_t)])
    outs = []
    for _ in range(3):
        T, S, Q = plan.run(O_t, D_t, P_t)
        torch.cuda.synchronize()
        outs.append((T.clone(), S.clone(), Q.clone()))
    for T, S, Q in outs[1:]:
        assert torch.equal(T, outs[0][0]) and torch.equal(S, outs[0][1]) and torch.equal(Q, outs[0][2])


def test_invalid_graph_reported(hip_device):
    # indices outside [0, n) are reported through the device status word
    import paper_2501_06872_amd as gt
    n = 5000
    O = np.arange(0, 4 * n + 1, 4, dtype=np.int64)
    rng = np.random.default_rng(1)
    D = rng.integers(0, n, size=4 * n).astype(np.int32)
    D[123] = n          # one past the end
    D[4567] = -1
    say("[case] invalid indices")
    _, _, _, st, _ = gpu_transpose(O, D, None, hip_device)
    assert st == gt.GT_ERR_INVALID_GRAPH
    # bad offsets with validation on
    O2 = O.copy()
    O2[10] = O2[11] + 1
    D2 = rng.integers(0, n, size=4 * n).astype(np.int32)
    say("[case] invalid offsets, validate=1")
    _, _, _, st, _ = gpu_transpose(O2, D2, None, hip_device, validate=True)
    assert st == gt.GT_ERR_INVALID_GRAPH


@pytest.mark.parametrize("payload", [False, True])
@pytest.mark.parametrize("validate", [False, True])
def test_invalid_ids_in_a_big_last_bin_stay_in_bounds(hip_device, payload, validate):
    """Destinations in [n, 2^ceil(log2 n)) and negative ones (whose masked
    digits alias into that range) inside a last bin longer than one k_final
    item: the graph is reported invalid and no write leaves the outputs
    (canary words after S, Q and T stay untouched)."""
    import paper_2501_06872_amd as gt
    n, m = 1000, 16000
    rng = np.random.default_rng(3)
    O = np.linspace(0, m, n + 1).astype(np.int64)
    cases = (("heuristic plan (one bin of 512..1023)", rng.integers(512, 1024, size=m), {}),
             ("fixed plan, 16-vertex bins", rng.integers(1000, 1024, size=m),
              dict(policy=gt.POLICY_FIXED, fine_bits=4, digit_bits=4)))
    for label, D, opt in cases:
        D = D.astype(np.int32)
        D[::97] = -1
        for u in range(n):
            D[O[u]:O[u + 1]].sort()
        assert np.count_nonzero(D >= n) + np.count_nonzero(D < 0) > 8192 // 16
        # the premise: the last bin (digits masked to 10 bits, as the
        # kernels see them) is longer than one 8192-edge k_final item
        fb = opt.get("fine_bits", 9)
        assert np.bincount((D.astype(np.int64) & 1023) >> fb).max() > 8192
        P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32) if payload else None
        say(f"[case] invalid ids in a big last bin: {label}, payload={payload}, validate={validate}")
        O_t, D_t, P_t = to_dev(O, D, P, hip_device)
        canary = 0x5A5A5A5A
        pad = 4096
        T_big = torch.full((n + 1 + pad,), canary, dtype=torch.int64, device=hip_device)
        S_big = torch.full((m + pad,), canary, dtype=torch.int32, device=hip_device)
        Q_big = torch.full((m + pad,), canary, dtype=torch.int32, device=hip_device) if payload else None
        out = (T_big[:n + 1], S_big[:m], Q_big[:m] if payload else None)
        plan = gt.Plan([(O_t, D_t, P_t)], gt.make_options(validate=validate, **opt))
        say("  params", plan.params())
        plan.run(O_t, D_t, P_t, out=out)
        torch.cuda.synchronize()
        assert plan.device_status() == gt.GT_ERR_INVALID_GRAPH
        assert bool((T_big[n + 1:] == canary).all()), "write past T"
        assert bool((S_big[m:] == canary).all()), "write past S"
        if payload:
            assert bool((Q_big[m:] == canary).all()), "write past Q"


def test_counter_check_quiet_on_valid_graphs(hip_device):
    # the digit-total and big-bin count checks raise no overflow on valid input
    import paper_2501_06872_amd as gt
    O, D, P = gen.rmat(18, 16, seed=5, permute=False)
    say("[case] counter checks on rmat18 (natural order: many big bins)")
    T, S, Q, st, params = gpu_transpose(O, D, P, hip_device)
    assert st == gt.GT_OK


@pytest.mark.parametrize("permute,payload", [(False, False), (True, True)])
def test_csc_input_transposes_back_to_the_csr(hip_device, permute, payload):
    """The CSC representations of Section V-A: the GPU's own CSC of an R-MAT
    scale-18 graph (natural order, and randomly relabelled with a payload),
    given back to the library as input (CSC -> CSR), returns the generated
    CSR exactly (its lists ascend, multi-edges in generation order), and both
    directions equal the oracle's."""
    import paper_2501_06872_amd as gt
    O, D, P = gen.rmat(18, 16, seed=18, permute=permute, payload=payload)
    label = f"rmat18{'p' if permute else ''} CSC input"
    say(f"[case] {label}: n={O.size - 1} m={D.size} payload={payload}")
    T, S, Q, st, _ = gpu_transpose(O, D, P, hip_device)
    assert st == gt.GT_OK
    rT, rS, rQ = oracle.transpose(O, D, P)
    assert np.array_equal(T, rT) and np.array_equal(S, rS)
    if payload:
        assert np.array_equal(Q, rQ)
    # the CSC as input: offsets T, "destinations" S, payload Q
    T2, S2, Q2, st2, _ = gpu_transpose(T, S, Q, hip_device)
    assert st2 == gt.GT_OK
    assert np.array_equal(T2, O), f"{label}: offsets do not return"
    assert np.array_equal(S2, D), f"{label}: lists do not return"
    if payload:
        assert np.array_equal(Q2, P), f"{label}: payload does not return"
    oT, oS, oQ = oracle.transpose(T, S, Q)
    assert np.array_equal(T2, oT) and np.array_equal(S2, oS)
    if payload:
        assert np.array_equal(Q2, oQ)


@pytest.mark.parametrize("variant", [1, 3, 4])
def test_first_pass_tile_counts(hip_device, variant):
    """Every partition pass places each tile with the column prefix of
    per-tile digit counts (16-bit per tile and digit; k_hist's for the first
    pass, k_tile_hist's over the previous pass's keys for a later one): a
    tile whose edges all share one digit (the largest count a tile can
    hold), edge counts around whole tiles and a ragged last tile, one pass,
    two passes (packed 16-bit keys between them) and three (32-bit keys)."""
    tile = {1: 8192, 3: 4096, 4: 16384}[variant]
    rng = np.random.default_rng(variant)
    for m in (1, 3, tile - 1, tile, tile + 1, 3 * tile + 5):
        n = 5000
        O = np.sort(rng.integers(0, m + 1, size=n + 1)).astype(np.int64)
        O[0], O[-1] = 0, m
        D = np.full(m, 4999, dtype=np.int32)  # every edge into one vertex: one digit per pass
        if m != tile:  # a whole tile of one digit stays: its count is the tile size
            D[::7] = rng.integers(0, n, size=D[::7].size)
        for u in range(n):
            D[O[u]:O[u + 1]].sort()
        for fb, db, passes in ((9, 9, 1), (4, 5, 2), (2, 4, 3)):
            params = assert_parity(O, D, None, hip_device, f"tile counts variant {variant} m={m} fine={fb} digit={db}",
                                   policy=1, fine_bits=fb, digit_bits=db, variant=variant)
            assert params["passes"] == passes, params
