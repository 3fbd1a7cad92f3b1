"""GPU: the persistent batched kernel (GT_FLAG_PERSISTENT), one launch that
drains a device work queue of every graph's phases, against the oracle:
eager, with payloads, empty and single-pass graphs, offsets validation, the
learned policy, back-to-back calls, replays of a captured HIP graph, and an
invalid graph in a batch (reported, every write inside its outputs); and
plans whose learned choice is made on the device (GT_FLAG_DEVICE_PLAN),
eagerly and captured together with the transposition.
Every case prints its name first."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def batch(count=24, seed=41, shift=6):
    """Uneven batch (sizes 2^10 .. 2^16 after the shift), plus an empty
    graph, a graph without edges, a one-vertex graph with self loops, a small
    graph that needs a single partition pass and two that need two."""
    specs = gen.batch_specs(count, seed=seed)
    for s in specs:
        s["n"] = max(1024, s["n"] >> shift)
    host = [gen.from_spec(s) for s in specs]
    host.append((np.zeros(1, np.int64), np.zeros(0, np.int32), None))                 # n = 0
    host.append((np.zeros(6, np.int64), np.zeros(0, np.int32), None))                 # n = 5, m = 0
    host.append((np.array([0, 3], np.int64), np.zeros(3, np.int32),
                 np.array([7, 8, 9], np.uint32)))                                     # n = 1, m = 3
    host.append(gen.generate(gen.FAM_UNIFORM, 700, 6, seed=3, payload=True))  # one pass
    # two partition passes (2^20 vertices, average degree 4)
    host.append(gen.generate(gen.FAM_RMAT, 1 << 20, 4, seed=5, permute=True, payload=True))
    host.append(gen.generate(gen.FAM_GEOMETRIC, 1 << 20, 4, seed=6))
    return host


def to_dev(O, D, P, dev):
    return (torch.from_numpy(O).to(dev), torch.from_numpy(D).to(dev),
            torch.from_numpy(P.view(np.int32)).to(dev) if P is not None else None)


def check(outs, host):
    for i, ((T, S, Q), (O, D, P)) in enumerate(zip(outs, host)):
        rT, rS, rQ = oracle.transpose(O, D, P)
        assert np.array_equal(T.cpu().numpy(), rT), f"graph {i}: offsets"
        assert np.array_equal(S.cpu().numpy(), rS), f"graph {i}: sources"
        if P is not None:
            assert np.array_equal(Q.cpu().numpy().view(np.uint32), rQ), f"graph {i}: payload"


def persistent_plan(gt, dev, **kw):
    flags = kw.pop("flags", 0) | gt.FLAG_PERSISTENT
    plan = gt.Plan(dev, gt.make_options(flags=flags, **kw))
    for i in range(len(dev)):
        p = plan.params(i)
        if dev[i][1].numel() > 0 and dev[i][0].numel() > 1:
            assert p["variant"] == 1 and p["digit_bits"] <= 9 and p["passes"] <= 2, (i, p)
    return plan


@pytest.mark.parametrize("validate", [False, True])
def test_persistent_eager_matches_oracle(hip_device, validate):
    import paper_2501_06872_amd as gt
    host = batch()
    say(f"[case] persistent batched eager, {len(host)} graphs, validate={validate}")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = persistent_plan(gt, dev, validate=validate)
    assert any(plan.params(i)["passes"] == 1 for i in range(len(dev)) if dev[i][1].numel() > 0)
    assert any(plan.params(i)["passes"] == 2 for i in range(len(dev)))
    outs = plan.run_batched(dev)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    check(outs, host)


def test_persistent_back_to_back(hip_device):
    """Two calls without a synchronisation between them, into different
    outputs: the second waits for the first call's copy of its tables."""
    import paper_2501_06872_amd as gt
    host = batch(12, seed=43)
    say(f"[case] persistent batched, two calls back to back, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = persistent_plan(gt, dev)
    a = plan.run_batched(dev)
    b = plan.run_batched(dev)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    check(a, host)
    check(b, host)


def test_persistent_mlp_policy(hip_device):
    import paper_2501_06872_amd as gt
    from paper_2501_06872_amd import mlp_model
    host = batch(16, seed=47, shift=4)
    say(f"[case] persistent batched, learned policy, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = persistent_plan(gt, dev, policy=gt.POLICY_MLP, model_path=mlp_model.DEFAULT_PATH)
    outs = plan.run_batched(dev)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    check(outs, host)


def test_persistent_graph_replay(hip_device):
    import paper_2501_06872_amd as gt
    host = batch(16, seed=45)
    say(f"[case] persistent batched, hipGraph replay, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = persistent_plan(gt, dev)
    outs = [plan.alloc_out(i, g[2].dtype if g[2] is not None else None) for i, g in enumerate(dev)]
    plan.run_batched(dev, outs)
    torch.cuda.synchronize()
    check(outs, host)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run_batched(dev, outs)
    for rep in range(3):
        for T, S, Q in outs:  # scribble over the outputs between replays
            T.fill_(-7)
            S.fill_(-7)
            if Q is not None:
                Q.fill_(7)
        junk = torch.randn(1 << 20, device=hip_device).sum()  # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        assert plan.device_status() == 0
        check(outs, host)
        del junk


def test_persistent_refuses_wide_status(hip_device):
    import paper_2501_06872_amd as gt
    host = batch(2, seed=49)
    say("[case] persistent plan with 64-bit look-back words is refused")
    dev = [to_dev(*g, hip_device) for g in host]
    with pytest.raises(gt.GTError) as e:
        gt.Plan(dev, gt.make_options(flags=gt.FLAG_PERSISTENT | gt.FLAG_WIDE_STATUS))
    assert e.value.status == gt.GT_ERR_UNSUPPORTED


@pytest.mark.parametrize("validate", [False, True])
def test_persistent_invalid_ids_stay_in_bounds(hip_device, validate):
    """A batch of an invalid graph (destinations in [n, 1024) and negative
    ones inside a last bin longer than one k_final item) and a valid one,
    as one persistent launch: the batch is reported invalid, no write leaves
    the invalid graph's outputs (canary words after T, S and Q), and the
    valid graph is still transposed exactly."""
    import paper_2501_06872_amd as gt
    n, m = 1000, 16000
    rng = np.random.default_rng(3)
    O = np.linspace(0, m, n + 1).astype(np.int64)
    D = rng.integers(512, 1024, size=m).astype(np.int32)
    D[::97] = -1
    for u in range(n):
        D[O[u]:O[u + 1]].sort()
    assert np.bincount((D.astype(np.int64) & 1023) >> 9).max() > 8192  # the premise: a big last bin
    P = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    good = gen.rmat(12, 8, seed=9)
    say(f"[case] persistent batch with invalid ids in a big last bin, validate={validate}")
    dev = [to_dev(O, D, P, hip_device), to_dev(*good, hip_device)]
    plan = persistent_plan(gt, dev, validate=validate)
    canary = 0x5A5A5A5A
    pad = 4096
    T_big = torch.full((n + 1 + pad,), canary, dtype=torch.int64, device=hip_device)
    S_big = torch.full((m + pad,), canary, dtype=torch.int32, device=hip_device)
    Q_big = torch.full((m + pad,), canary, dtype=torch.int32, device=hip_device)
    outs = [(T_big[:n + 1], S_big[:m], Q_big[:m]), plan.alloc_out(1, None)]
    plan.run_batched(dev, outs)
    torch.cuda.synchronize()
    assert plan.device_status() == gt.GT_ERR_INVALID_GRAPH
    assert bool((T_big[n + 1:] == canary).all()), "write past T"
    assert bool((S_big[m:] == canary).all()), "write past S"
    assert bool((Q_big[m:] == canary).all()), "write past Q"
    check(outs[1:], [good])


def device_plan_options(gt):
    from paper_2501_06872_amd import mlp_model
    return gt.make_options(policy=gt.POLICY_MLP, model_path=mlp_model.DEFAULT_PATH,
                           flags=gt.FLAG_PERSISTENT | gt.FLAG_DEVICE_PLAN)


def check_device_choices(plan, dev):
    learned = 0
    for i in range(len(dev)):
        c = plan.device_choice(i)
        assert c["variant"] == 1 and 4 <= c["digit_bits"] <= 9 and -1 <= c["config"] < 32, (i, c)
        learned += c["config"] >= 0
    return learned


def test_device_plan_matches_oracle(hip_device):
    """The learned choice made on the device (sampling, network, argmin in
    kernels), every graph laid out and the queue built by the planning
    kernel: outputs against the oracle."""
    import paper_2501_06872_amd as gt
    host = batch(16, seed=51, shift=4)
    say(f"[case] device-planned persistent batch, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = gt.Plan(dev, device_plan_options(gt))
    outs = plan.run_batched(dev)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    check(outs, host)
    learned = check_device_choices(plan, dev)
    say(f"  {learned} of {len(dev)} graphs took the network's choice")
    assert learned > 0
    outs2 = plan.run_batched(dev)  # a second call: the same choices, laid out again
    torch.cuda.synchronize()
    check(outs2, host)


def test_device_plan_and_transpose_in_one_captured_graph(hip_device):
    """gt_plan (device plan) and gt_transpose_batched captured together in one
    HIP graph, replayed three times with scribbled outputs between."""
    import paper_2501_06872_amd as gt
    host = batch(12, seed=53, shift=5)
    say(f"[case] device plan + persistent batch captured together, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    outs = [(torch.empty(g[0].numel(), dtype=torch.int64, device=hip_device),
             torch.empty(g[1].numel(), dtype=torch.int32, device=hip_device),
             torch.empty(g[1].numel(), dtype=g[2].dtype, device=hip_device) if g[2] is not None else None)
            for g in dev]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, capture_error_mode="relaxed"):
        plan = gt.Plan(dev, device_plan_options(gt))
        plan.run_batched(dev, outs)
    for rep in range(3):
        for T, S, Q in outs:
            T.fill_(-7)
            S.fill_(-7)
            if Q is not None:
                Q.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        assert plan.device_status() == 0
        check(outs, host)
    assert check_device_choices(plan, dev) > 0
