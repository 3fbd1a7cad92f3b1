"""GPU: a HEURISTIC plan and its transposition captured together in one HIP
graph (planning does no device work and no synchronisation), replayed
several times with unrelated eager work in between, each replay checked bit
for bit against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("payload", [False, True])
def test_plan_and_transpose_in_one_captured_graph(hip_device, payload):
    import paper_2501_06872_amd as gt
    L = gt.lib()
    O, D, P = gen.rmat(17, 16, seed=9, permute=True, payload=payload)
    say(f"[case] plan + transpose captured, rmat17p payload={payload}")
    rT, rS, rQ = oracle.transpose(O, D, P)
    O_t = torch.from_numpy(O).to(hip_device)
    D_t = torch.from_numpy(D).to(hip_device)
    P_t = torch.from_numpy(P.view(np.int32)).to(hip_device) if P is not None else None
    csr = gt._csr(O_t, D_t, P_t)
    size = ctypes.c_size_t()
    assert L.gt_workspace_size(ctypes.byref(csr), 1, ctypes.byref(size)) == gt.GT_OK
    ws = torch.empty(size.value, dtype=torch.uint8, device=hip_device)
    n, m = O.size - 1, D.size
    T = torch.empty(n + 1, dtype=torch.int64, device=hip_device)
    S = torch.empty(m, dtype=torch.int32, device=hip_device)
    Q = torch.empty(m, dtype=torch.int32, device=hip_device) if payload else None
    csc = gt.CSC(T.data_ptr(), S.data_ptr(), Q.data_ptr() if Q is not None else None)
    opts = gt.make_options(policy=gt.POLICY_HEURISTIC)
    h = ctypes.c_void_p()
    side = torch.cuda.Stream(device=hip_device)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        s = ctypes.c_void_p(torch.cuda.current_stream(hip_device).cuda_stream)
        rc_plan = L.gt_plan(ctypes.byref(csr), 1, ctypes.byref(opts), None, 0, s, ctypes.byref(h))
        rc_run = L.gt_transpose(h, ctypes.byref(csr), ctypes.byref(csc), ws.data_ptr(), size.value, s) \
            if rc_plan == gt.GT_OK else -1
    assert rc_plan == gt.GT_OK and rc_run == gt.GT_OK, (rc_plan, rc_run)
    try:
        for rep in range(3):
            T.fill_(-7)
            S.fill_(-7)
            if Q is not None:
                Q.fill_(7)
            junk = torch.randn(1 << 20, device=hip_device).sum()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            say(f"  replay {rep}")
            assert L.gt_plan_device_status(h, ws.data_ptr()) == gt.GT_OK
            assert np.array_equal(T.cpu().numpy(), rT)
            assert np.array_equal(S.cpu().numpy(), rS)
            if payload:
                assert np.array_equal(Q.cpu().numpy().view(np.uint32), rQ)
            del junk
    finally:
        L.gt_plan_destroy(h)
