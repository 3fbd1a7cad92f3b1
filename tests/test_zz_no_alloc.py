"""gt_transpose_noalloc (the library's static scratch instead of a caller
workspace) against gt_transpose on the same graphs: bit-exact outputs on two
calls in a row, the second on a smaller graph, plus the device status word
it hands back."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _dev(O, D, P, dev):
    return (torch.from_numpy(O).to(dev), torch.from_numpy(D).to(dev),
            torch.from_numpy(P.view(np.int32)).to(dev) if P is not None else None)


def _run_both(gt, O, D, P, dev):
    O_t, D_t, P_t = _dev(O, D, P, dev)
    plan = gt.Plan([(O_t, D_t, P_t)])
    assert plan.workspace_size() <= gt.NOALLOC_SCRATCH_BYTES
    ref = plan.run(O_t, D_t, P_t)
    # outputs prefilled with a pattern, so a slot the call leaves unwritten shows
    out = tuple(torch.full_like(x, 0x3C3C3C3C) if x is not None else None for x in plan.alloc_out(
        0, P_t.dtype if P_t is not None else None))
    status = torch.full((1,), 0x7F, dtype=torch.int32, device=dev)
    plan.run_noalloc(O_t, D_t, P_t, out, status)
    torch.cuda.synchronize()
    assert plan.device_status() == gt.GT_OK
    return ref, out, int(status.item())


def test_noalloc_matches_workspace_entry_point(hip_device):
    import paper_2501_06872_amd as gt
    cases = (("rmat16 natural order, payload", gen.rmat(16, 16, seed=1, permute=False, payload=True)),
             ("rmat12 permuted, no payload", gen.rmat(12, 8, seed=7, permute=True, payload=False)))
    for label, (O, D, P) in cases:
        say(f"[case] noalloc vs gt_transpose: {label}, n={O.size - 1} m={D.size}")
        ref, out, st = _run_both(gt, O, D, P, hip_device)
        assert st == 0, f"status word {st:#x}"
        for name, a, b in zip("TSQ", ref, out):
            if a is None:
                assert b is None
                continue
            assert torch.equal(a, b), f"{name} differs from gt_transpose"
        rT, rS, rQ = oracle.transpose(O, D, P)
        assert np.array_equal(out[0].cpu().numpy(), rT)
        assert np.array_equal(out[1].cpu().numpy(), rS)
        if P is not None:
            assert np.array_equal(out[2].cpu().numpy().view(np.uint32), rQ)


def test_noalloc_reports_invalid_graph_and_refuses_big_plans(hip_device):
    import paper_2501_06872_amd as gt
    rng = np.random.default_rng(11)
    n = 3000
    O = np.linspace(0, 8 * n, n + 1).astype(np.int64)
    D = rng.integers(0, n, size=8 * n).astype(np.int32)
    D[77] = n  # one past the last vertex
    say("[case] noalloc: an index outside [0, n) sets the status word")
    O_t, D_t, _ = _dev(O, D, None, hip_device)
    plan = gt.Plan([(O_t, D_t, None)])
    out = plan.alloc_out(0)
    status = torch.zeros(1, dtype=torch.int32, device=hip_device)
    plan.run_noalloc(O_t, D_t, None, out, status)
    torch.cuda.synchronize()
    assert int(status.item()) & 1
    # then a valid graph again: the shared scratch starts from a clear status
    O2, D2, _ = gen.rmat(10, 4, seed=3, permute=True, payload=False)
    say("[case] noalloc after an invalid graph: a valid one reports 0")
    ref, out2, st = _run_both(gt, O2, D2, None, hip_device)
    assert st == 0
    assert all(torch.equal(a, b) for a, b in zip(ref[:2], out2[:2]))
    # a plan whose workspace exceeds the scratch is refused before any launch
    n3, m3 = 1 << 20, 1 << 24
    O3 = torch.zeros(n3 + 1, dtype=torch.int64, device=hip_device)
    O3[-1] = m3
    D3 = torch.zeros(m3, dtype=torch.int32, device=hip_device)
    plan3 = gt.Plan([(O3, D3, None)])
    assert plan3.workspace_size() > gt.NOALLOC_SCRATCH_BYTES
    say("[case] noalloc refuses a plan needing more than the scratch")
    with pytest.raises(gt.GTError) as ei:
        plan3.run_noalloc(O3, D3, None, plan3.alloc_out(0))
    assert ei.value.status == gt.GT_ERR_WORKSPACE_TOO_SMALL
