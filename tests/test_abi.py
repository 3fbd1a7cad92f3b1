"""The C ABI library loads and exports every entry point include/gt.h declares
(no GPU calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gt.h")
LIB = os.path.join(ROOT, "paper_2501_06872_amd", "libgt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("gt_plan", "gt_transpose", "gt_transpose_batched", "gt_workspace_size", "gt_plan_destroy",
              "gt_status_string", "gt_device_status", "gt_plan_device_status"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for f in declared_functions():
        assert hasattr(lib, f), f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgt.so not built")
def test_status_strings_and_argument_errors_without_gpu():
    import paper_2501_06872_amd as gt
    L = gt.lib()
    assert gt.status_string(0) == "ok"
    assert "workspace" in gt.status_string(3)
    # argument checks happen on the host, before any device call
    size = ctypes.c_size_t()
    assert L.gt_workspace_size(None, 1, ctypes.byref(size)) == gt.GT_ERR_INVALID_ARGUMENT
    bad = gt.CSR(-1, 0, 1, None, None)
    assert L.gt_workspace_size(ctypes.byref(bad), 1, ctypes.byref(size)) == gt.GT_ERR_INVALID_ARGUMENT
    big = gt.CSR(1 << 31, 0, 1, None, None)  # n beyond int32 IDs
    assert L.gt_workspace_size(ctypes.byref(big), 1, ctypes.byref(size)) == gt.GT_ERR_INVALID_ARGUMENT
    ok = gt.CSR(1000, 16000, 1, 1, None)
    assert L.gt_workspace_size(ctypes.byref(ok), 1, ctypes.byref(size)) == gt.GT_OK and size.value > 0
    h = ctypes.c_void_p()
    opts = gt.make_options(policy=gt.POLICY_FIXED, fine_bits=12)
    assert L.gt_plan(ctypes.byref(ok), 1, ctypes.byref(opts), None, 0, None, ctypes.byref(h)) == \
        gt.GT_ERR_UNSUPPORTED
    assert L.gt_transpose(None, None, None, None, 0, None) == gt.GT_ERR_INVALID_ARGUMENT
    # more than 2^32 edges: refused before any device work
    huge = gt.CSR(1 << 28, (1 << 32) + 1, 1, 1, None)
    assert L.gt_workspace_size(ctypes.byref(huge), 1, ctypes.byref(size)) == gt.GT_ERR_UNSUPPORTED
    assert L.gt_plan(ctypes.byref(huge), 1, None, None, 0, None, ctypes.byref(h)) == gt.GT_ERR_UNSUPPORTED
    at_limit = gt.CSR(1 << 28, 1 << 32, 1, 1, None)
    assert L.gt_workspace_size(ctypes.byref(at_limit), 1, ctypes.byref(size)) == gt.GT_OK
    assert gt.status_string(gt.GT_ERR_COUNTER_OVERFLOW) == "counter overflow"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgt.so not built")
def test_heuristic_and_fixed_plans_do_no_device_work():
    """There is no GPU in this process: a plan that touched the device
    (sampling, a synchronisation) would fail.  HEURISTIC (the default, no
    options) and FIXED plans succeed with no workspace and no stream."""
    import paper_2501_06872_amd as gt
    L = gt.lib()
    g = gt.CSR(1 << 26, 1 << 30, 1, 1, None)
    for opts in (None, gt.make_options(policy=gt.POLICY_HEURISTIC),
                 gt.make_options(policy=gt.POLICY_FIXED, fine_bits=8, digit_bits=9)):
        h = ctypes.c_void_p()
        rc = L.gt_plan(ctypes.byref(g), 1, ctypes.byref(opts) if opts is not None else None, None, 0, None,
                       ctypes.byref(h))
        assert rc == gt.GT_OK
        out = [ctypes.c_int32() for _ in range(4)]
        assert L.gt_plan_params(h, 0, *[ctypes.byref(x) for x in out]) == gt.GT_OK
        assert out[2].value == 2  # two partition passes at 2^26 vertices
        assert L.gt_plan_device_status(None, None) == gt.GT_ERR_INVALID_ARGUMENT
        assert L.gt_plan_destroy(h) == gt.GT_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgt.so not built")
def test_every_config_plans_a_tile_variant_that_has_an_instance():
    """Planning is host-only for the fixed policy.  The 16-wave tile variants
    (2 and 4) have no instance for 10-bit digits: a plan that needs 10-bit
    digits must run the 8-wave x 16-edge tile (variant 1) for every pass, so
    the tile size its buffers were sized for is the one the kernels use."""
    import paper_2501_06872_amd as gt
    L = gt.lib()
    seen_fallback = False
    for n, m, pay in ((97484, 389936, 1), (1 << 17, 1 << 20, None), ((1 << 20) + 3, 1 << 23, 1),
                      (1 << 26, 1 << 30, None), (5993, 95888, 1)):
        g = gt.CSR(n, m, 1, 1, pay)
        for c in range(gt.num_configs()):
            cfg = gt.config(c)
            fb, db, v = cfg["fine_bits"], cfg["digit_bits"], cfg["variant"]
            h = ctypes.c_void_p()
            opts = gt.make_options(policy=gt.POLICY_FIXED, fine_bits=fb, digit_bits=db, variant=v)
            assert L.gt_plan(ctypes.byref(g), 1, ctypes.byref(opts), None, 0, None, ctypes.byref(h)) == gt.GT_OK
            out = [ctypes.c_int32() for _ in range(4)]
            assert L.gt_plan_params(h, 0, *[ctypes.byref(x) for x in out]) == gt.GT_OK
            pfb, pdb, passes, pv = (x.value for x in out)
            assert 1 <= passes <= 3 and 1 <= pdb <= 10 and pv in (1, 2, 3, 4)
            if pdb == 10:
                assert pv in (1, 3), (n, c, pdb, pv)
                seen_fallback |= v in (2, 4)
            else:
                assert pv == v, (n, c, pdb, pv)
            assert L.gt_plan_destroy(h) == gt.GT_OK
    assert seen_fallback
