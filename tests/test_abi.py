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
              "gt_status_string", "gt_device_status"):
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
