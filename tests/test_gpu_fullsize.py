"""GPU: whole-output parity at the full workload sizes.

Every offset, every source and every payload word of the transposition is
compared with the oracle's (Algorithm 1 run by one thread, whose lists come
out in increasing CSR edge position), on each synthetic workload at its
stated size, in the launch configuration the benchmark times (a heuristic
plan, one gt_transpose): R-MAT scale 24 with permuted IDs and a float32
payload, uniform and geometric-locality graphs of 2^26 vertices and 2^30
edges, R-MAT scale 26 in natural and permuted order, and R-MAT scale 28
(2^32 edges: 64-bit look-back words, three partition passes).  Then the
512-graph uneven batch, planned by the learned policy and replayed from a
captured HIP graph, over the internal streams and as one launch of the
persistent kernel.  Each case prints its name and its steps as it goes."""
import time

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print(*a, flush=True)


def _check_whole(label, O, D, P, T, S, Q):
    t0 = time.time()
    rT, rS, rQ = oracle.transpose(O, D, P)
    say(f"  {label}: oracle {time.time() - t0:.1f} s")
    assert np.array_equal(T, rT), f"{label}: offsets differ"
    del rT
    assert np.array_equal(S, rS), f"{label}: sources differ"
    del rS
    if P is not None:
        assert np.array_equal(Q.view(np.uint32), rQ), f"{label}: payload differs"


@pytest.mark.parametrize("workload", ["rmat24p", "uniform26", "geom26", "rmat26", "rmat26p", "rmat28p"])
def test_full_size_matches_oracle(hip_device, workload):
    import paper_2501_06872_amd as gt
    t0 = time.time()
    O, D, P = gen.workload(workload)
    n, m = O.size - 1, D.size
    say(f"[case] full size {workload}: n={n} m={m} payload={P is not None}, generated in {time.time() - t0:.1f} s")
    O_t = torch.from_numpy(O).to(hip_device)
    D_t = torch.from_numpy(D).to(hip_device)
    P_t = torch.from_numpy(P.view(np.int32)).to(hip_device) if P is not None else None
    plan = gt.Plan([(O_t, D_t, P_t)])
    say(f"  params {plan.params()} packed={plan.packed()}")
    T_t, S_t, Q_t = plan.run(O_t, D_t, P_t)
    torch.cuda.synchronize()
    assert plan.device_status() == gt.GT_OK
    del O_t, D_t, P_t, plan
    T = T_t.cpu().numpy()
    S = S_t.cpu().numpy()
    Q = Q_t.cpu().numpy() if Q_t is not None else None
    del T_t, S_t, Q_t
    torch.cuda.empty_cache()
    say(f"  transposed and copied back in {time.time() - t0:.1f} s")
    _check_whole(workload, O, D, P, T, S, Q)
    say(f"  {workload}: bit-exact, {time.time() - t0:.1f} s in all")


@pytest.mark.parametrize("launcher", ["lanes", "persistent"])
def test_batch512_learned_plan_graph_replay_matches_oracle(hip_device, launcher):
    import paper_2501_06872_amd as gt
    t0 = time.time()
    import concurrent.futures
    import os
    from paper_2501_06872_amd import mlp_model
    assert os.path.exists(mlp_model.DEFAULT_PATH), "the committed model"
    specs = gen.batch_specs(512, seed=5)
    with concurrent.futures.ThreadPoolExecutor(16) as pool:  # the generator releases the GIL
        host = list(pool.map(gen.from_spec, specs))
    m_total = sum(int(g[1].size) for g in host)
    say(f"[case] batch512 (seed 5), {launcher}: 512 graphs, m={m_total}, generated in {time.time() - t0:.1f} s")
    dev = [(torch.from_numpy(O).to(hip_device), torch.from_numpy(D).to(hip_device),
            torch.from_numpy(P.view(np.int32)).to(hip_device) if P is not None else None) for O, D, P in host]
    flags = gt.FLAG_PERSISTENT if launcher == "persistent" else 0
    plan = gt.Plan(dev, gt.make_options(policy=gt.POLICY_MLP, model_path=mlp_model.DEFAULT_PATH, flags=flags))
    say(f"  MLP plan built, {time.time() - t0:.1f} s")
    outs = [plan.alloc_out(i, g[2].dtype if g[2] is not None else None) for i, g in enumerate(dev)]
    plan.run_batched(dev, outs)  # eager warm-up (creates the internal streams of the lanes)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run_batched(dev, outs)
    for T, S, Q in outs:  # scribble over the outputs, then replay
        T.fill_(-7)
        S.fill_(-7)
        if Q is not None:
            Q.fill_(7)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert plan.device_status() == gt.GT_OK
    say(f"  captured batch replayed, {time.time() - t0:.1f} s")
    for i, ((T, S, Q), (O, D, P)) in enumerate(zip(outs, host)):
        rT, rS, rQ = oracle.transpose(O, D, P)
        assert np.array_equal(T.cpu().numpy(), rT), f"graph {i}: offsets differ"
        assert np.array_equal(S.cpu().numpy(), rS), f"graph {i}: sources differ"
        if P is not None:
            assert np.array_equal(Q.cpu().numpy().view(np.uint32), rQ), f"graph {i}: payload differs"
        if i % 64 == 63:
            say(f"  {i + 1} graphs bit-exact, {time.time() - t0:.1f} s")
