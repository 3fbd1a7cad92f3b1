"""GPU: batched transposition of uneven graphs, eager and replayed from a
captured HIP graph, against the oracle.  Every case prints its name first."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def small_batch(count=24, seed=31):
    specs = gen.batch_specs(count, seed=seed)
    for s in specs:  # keep the test quick: sizes 2^10 .. 2^16
        s["n"] = max(1024, s["n"] >> 6)
    return specs, [gen.from_spec(s) for s in specs]


def to_dev(O, D, P, dev):
    return (torch.from_numpy(O).to(dev), torch.from_numpy(D).to(dev),
            torch.from_numpy(P.view(np.int32)).to(dev) if P is not None else None)


def check(outs, host):
    for (T, S, Q), (O, D, P) in zip(outs, host):
        rT, rS, rQ = oracle.transpose(O, D, P)
        assert np.array_equal(T.cpu().numpy(), rT)
        assert np.array_equal(S.cpu().numpy(), rS)
        if P is not None:
            assert np.array_equal(Q.cpu().numpy().view(np.uint32), rQ)


@pytest.mark.parametrize("policy", ["heuristic", "fixed"])
def test_batched_eager_matches_oracle(hip_device, policy):
    import paper_2501_06872_amd as gt
    specs, host = small_batch()
    say(f"[case] batched eager, {len(host)} graphs, policy {policy}")
    dev = [to_dev(*g, hip_device) for g in host]
    opts = gt.make_options(policy=gt.POLICY_HEURISTIC if policy == "heuristic" else gt.POLICY_FIXED)
    plan = gt.Plan(dev, opts)
    outs = plan.run_batched(dev)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    check(outs, host)


def test_batched_graph_replay(hip_device):
    import paper_2501_06872_amd as gt
    specs, host = small_batch(16, seed=33)
    say(f"[case] batched hipGraph replay, {len(host)} graphs")
    dev = [to_dev(*g, hip_device) for g in host]
    plan = gt.Plan(dev)
    outs = [plan.alloc_out(i, g[2].dtype if g[2] is not None else None) for i, g in enumerate(dev)]
    plan.run_batched(dev, outs)          # eager warm-up (creates the internal streams)
    torch.cuda.synchronize()
    check(outs, host)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run_batched(dev, outs)
    for rep in range(3):
        for T, S, Q in outs:             # scribble over the outputs between replays
            T.fill_(-7)
            S.fill_(-7)
            if Q is not None:
                Q.fill_(7)
        junk = torch.randn(1 << 20, device=hip_device).sum()  # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        check(outs, host)
        del junk
