"""Random-access microbenchmark on one MI355X and the performance models of
Eq. 2 and Eq. 3 (Section IV-B) with the per-access times it measures.

Fig. 3 (Section III-B) compares random reads, writes and atomic writes on
arrays that fit a cache level with arrays far larger than it.  Here the
levels are a workgroup's LDS, a few hot cache lines shared by every thread,
an array inside one XCD's L2, one inside the Infinity Cache and one in HBM;
every launch keeps about a million threads in flight.  Rates are accesses
per second over the whole GPU, and the per-access times of the models are
their inverses (the machine is throughput-bound, so an aggregate rate is
what a kernel of many independent accesses sees).

With --model the unordered strategies' Step 1 (the in-degree count, HLH and
Atomic GT) is timed on synthetic graphs and set against the models:
Eq. 2 is solved for the hit ratio h the Atomic count implies, Eq. 3 predicts
the HLH count from the exact coverage of the top-k destinations (k = 2048,
the HDV table's capacity), and the break-even coverage is where Eq. 3 meets
Eq. 2 at h = 0.

    python -m paper_2501_06872_amd.microbench [--model] [--workloads rmat24p,...]
        [--levels lds,hot,l2,mall,hbm] [--kinds read,write,atomic,index]

Prints a table on stderr and one JSON line on stdout.
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

import paper_2501_06872_amd as gt

LEVELS = {  # name: (memory, words)
    "lds": (gt.MEMORY_LDS, 8192),        # 32 KB per workgroup, private to it
    "hot": (gt.MEMORY_GLOBAL, 64),       # 256 B: two cache lines shared by all threads
    "l2": (gt.MEMORY_GLOBAL, 1 << 18),   # 1 MB, inside one XCD's 4 MB L2
    "mall": (gt.MEMORY_GLOBAL, 1 << 25),  # 128 MB, inside the 256 MB Infinity Cache
    "hbm": (gt.MEMORY_GLOBAL, 1 << 31),  # 8 GB
}
KINDS = {"read": gt.ACCESS_READ, "write": gt.ACCESS_WRITE, "atomic": gt.ACCESS_ATOMIC, "index": gt.ACCESS_INDEX}
BLOCKS = 4096  # 2^20 threads
HDV_K = 2048


def _time_launch(buf, words, kind, memory, per, sink):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    gt.random_access(buf, words, kind, memory, 1234, per, BLOCKS, sink)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def measure(level, kind_name, dev, target_ms=20.0, reps=3):
    """Accesses per second (whole GPU) for one level and kind: the median of
    `reps` launches sized to take about target_ms each."""
    memory, words = LEVELS[level]
    kind = KINDS[kind_name]
    size = words * (BLOCKS if memory == gt.MEMORY_LDS else 1)
    buf = torch.zeros(size, dtype=torch.int32, device=dev)
    sink = torch.empty(BLOCKS * gt.THREADS_PER_BLOCK, dtype=torch.int32, device=dev)
    _time_launch(buf, words, kind, memory, 16, sink)
    probe = max(_time_launch(buf, words, kind, memory, 64, sink), 1e-3)
    per = int(min(max(64 * target_ms / probe, 16), 1 << 16))
    ms = sorted(_time_launch(buf, words, kind, memory, per, sink) for _ in range(reps))[reps // 2]
    del buf, sink
    return BLOCKS * gt.THREADS_PER_BLOCK * per / (ms * 1e-3), per, ms


def count_step_ms(O_t, D_t, P_t, strategy, steps=3):
    """Average time of the unordered strategy's Step 1 kernel (k_hlh_count)."""
    plan = gt.Plan([(O_t, D_t, P_t)], gt.make_options(strategy=strategy))
    out = plan.alloc_out(0, P_t.dtype if P_t is not None else None)
    plan.run(O_t, D_t, P_t, out=out)
    torch.cuda.synchronize()
    plan.profile(True)
    for _ in range(steps):
        plan.run(O_t, D_t, P_t, out=out)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    total, launches = prof["k_hlh_count"]
    return total / launches


def model(workloads, rates, dev):
    import gen
    ps = {key: 1e12 / r for key, r in rates.items()}  # picoseconds per access, whole GPU
    t_aw_m, t_aw_h = ps[("hbm", "atomic")], ps[("l2", "atomic")]
    t_w_h, t_r_h = ps[("lds", "atomic")], ps[("lds", "read")]
    out = {"t_ps": {"aw_m (atomic, hbm)": t_aw_m, "aw_h (atomic, l2)": t_aw_h, "w_h (atomic, lds)": t_w_h,
                    "r_h (read, lds)": t_r_h},
           "break_even_coverage_h0": t_r_h / (t_aw_m - t_w_h) if t_aw_m > t_w_h else None,
           "graphs": []}
    for name in workloads:
        t0 = time.time()
        O, D, P = gen.workload(name)
        n, m = O.size - 1, D.size
        deg = np.bincount(D, minlength=n)
        k = min(HDV_K, n)
        coverage = float(np.partition(deg, n - k)[n - k:].sum()) / m
        del deg
        O_t, D_t = torch.from_numpy(O).to(dev), torch.from_numpy(D).to(dev)
        P_t = torch.from_numpy(P.view(np.int32)).to(dev) if P is not None else None
        del O, D, P
        atomic_ms = count_step_ms(O_t, D_t, P_t, gt.STRATEGY_ATOMIC)
        hlh_ms = count_step_ms(O_t, D_t, P_t, gt.STRATEGY_HLH)
        del O_t, D_t, P_t
        torch.cuda.empty_cache()
        per_edge_atomic = atomic_ms * 1e9 / m  # ps per edge
        per_edge_hlh = hlh_ms * 1e9 / m
        h = (t_aw_m - per_edge_atomic) / (t_aw_m - t_aw_h) if t_aw_m != t_aw_h else None
        pred_hlh = coverage * (t_w_h - t_aw_m) + t_aw_m + t_r_h
        row = {"workload": name, "m": m, "coverage_top2048": round(coverage, 4),
               "atomic_count_ms": round(atomic_ms, 3), "hlh_count_ms": round(hlh_ms, 3),
               "atomic_ps_per_edge": round(per_edge_atomic, 2), "hlh_ps_per_edge": round(per_edge_hlh, 2),
               "eq2_hit_ratio": round(h, 3) if h is not None else None,
               "eq3_hlh_ps_per_edge": round(pred_hlh, 2),
               "eq3_over_measured": round(pred_hlh / per_edge_hlh, 3)}
        out["graphs"].append(row)
        print(f"[model] {name}: {row} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--model", action="store_true", help="also fit Eq. 2 / Eq. 3 to the unordered Step 1")
    ap.add_argument("--workloads", default="rmat24p,rmat26,rmat26p,uniform26,geom26")
    ap.add_argument("--levels", default=",".join(LEVELS))
    ap.add_argument("--kinds", default=",".join(KINDS))
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the microbenchmark needs a GPU")
    dev = torch.device("cuda:0")
    levels = [lv for lv in args.levels.split(",") if lv]
    rates, detail = {}, {}
    kinds = [k for k in args.kinds.split(",") if k]
    for level in levels:
        for kind in kinds:
            r, per, ms = measure(level, kind, dev)
            rates[(level, kind)] = r
            detail[f"{level}/{kind}"] = {"g_per_s": round(r / 1e9, 2), "per_thread": per, "ms": round(ms, 3)}
            print(f"[rate] {level:5s} {kind:7s} {r / 1e9:10.2f} G/s  (per thread {per}, {ms:.2f} ms)",
                  file=sys.stderr, flush=True)
    base = rates.get(("l2", "read"))
    res = {"metric": "random accesses/s (G/s)", "threads": BLOCKS * gt.THREADS_PER_BLOCK,
           "levels": {k: list(v) for k, v in LEVELS.items() if k in levels}, "rates": detail,
           "normalised_to_l2_read": ({f"{lv}/{k}": round(r / base, 3) for (lv, k), r in rates.items()}
                                     if base else None)}
    if args.model:
        need = {("hbm", "atomic"), ("l2", "atomic"), ("lds", "atomic"), ("lds", "read")}
        if not need <= set(rates):
            raise SystemExit("--model needs the lds, l2 and hbm levels")
        res["model"] = model([w for w in args.workloads.split(",") if w], rates, dev)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
