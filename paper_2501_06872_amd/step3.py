"""Load balance of Step 3 of the unordered strategies (Section V-F).

``balance(stamps, hz)`` summarises the per-chunk wall-clock stamps that a
plan built with GT_FLAG_STEP3_TIMES records (one row per chunk workgroup:
start, own head done, end).  The imbalance is the paper's measure of Step 3:
(longest workgroup time - mean workgroup time) / longest workgroup time.
"""
import numpy as np


def balance(stamps, hz):
    st = np.asarray(stamps, dtype=np.float64)
    busy = (st[:, 2] - st[:, 0]) / hz
    head = (st[:, 1] - st[:, 0]) / hz
    span = (st[:, 2].max() - st[:, 0].min()) / hz
    longest = float(busy.max()) if busy.size else 0.0
    return {
        "workgroups": int(busy.size),
        "span_ms": 1e3 * float(span),
        "longest_ms": 1e3 * longest,
        "mean_ms": 1e3 * float(busy.mean()) if busy.size else 0.0,
        "head_mean_ms": 1e3 * float(head.mean()) if head.size else 0.0,
        "imbalance": (longest - float(busy.mean())) / longest if longest > 0 else 0.0,
    }
