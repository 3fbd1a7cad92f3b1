"""Summarise rocprofv3 runs of bench.py into profiles/gt_kernels_<workload>.txt.

    python -m paper_2501_06872_amd.profile_summary <workload> <passes> <dir>
    python -m paper_2501_06872_amd.profile_summary batch512 --batch <dir>
    python -m paper_2501_06872_amd.profile_summary random-read --fetch <dir> <per> <threads>

<dir> holds the three rocprofv3 databases of one workload, named as the
commands printed in the summary make them (trace_results.db,
fetch_results.db, write_results.db).  The summary gives per-kernel launch
counts and average durations (kernel trace), and HBM bytes per launch from
FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for the
1 GiB device copy that bench.py --calibrate makes.  It also records the
SHA-256 of the kernel sources, so that bench.py uses the traffic figures
only while the kernels are the ones profiled.
"""
import collections
import hashlib
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_2501_06872_amd/csrc/gt_kernels.hip", "paper_2501_06872_amd/csrc/gt_bodies.hpp",
                  "paper_2501_06872_amd/csrc/gt_device.hpp", "paper_2501_06872_amd/csrc/gt_internal.h")


def label(name, passes):
    m = re.match(r"void gt::k_lsd<(\d+), (\d+), (\d+), (true|false), (true|false), (true|false), "
                 r"(?:(?:true|false), )?(unsigned int|unsigned long)>", name)
    if m:
        csr_in, last = m.group(4) == "true", m.group(6) == "true"
        if csr_in:
            return "k_lsd_pass0"
        return f"k_lsd_pass{passes - 1}" if last else "k_lsd_pass1"
    m = re.match(r"(?:void )?gt::(k_[a-z0-9_]+)", name)
    if m:
        return m.group(1)
    if "copyBuffer" in name:
        return "copy (runtime blit)"
    if "FillFunctor" in name:
        return "torch fill"
    return name[:40]


def summarise(workload, passes, d):
    def q(db, sql):
        return sqlite3.connect(db).execute(sql).fetchall()
    tr = q(os.path.join(d, "trace_results.db"), "select dispatch_id, name, duration from kernels")
    pm = {}
    for tag, cn in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        pm[tag] = q(os.path.join(d, f"{tag}_results.db"),
                    f"select kernel_name, value, grid_size from counters_collection where counter_name='{cn}'")
    # calibration: the 1 GiB device copy (the largest copyBuffer dispatch)
    cf = max(v for k, v, g in pm["fetch"] if "copyBuffer" in k)
    cw = max(v for k, v, g in pm["write"] if "copyBuffer" in k)
    gib_kib = 1 << 20
    ffac, wfac = gib_kib / cf, gib_kib / cw
    copy_us = max(dur for _, n, dur in tr if "copyBuffer" in n) / 1000
    stats = collections.OrderedDict()
    for _, n, dur in tr:
        s = stats.setdefault(label(n, passes), [0, 0.0, n])
        s[0] += 1
        s[1] += dur
    agg = {}
    for tag in ("fetch", "write"):
        acc = collections.defaultdict(list)
        for k, v, g in pm[tag]:
            acc[label(k, passes)].append(v)
        agg[tag] = {k: sum(v) / len(v) for k, v in acc.items()}
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    cmd = f"python3 bench.py --workload {workload} --steps 5 --warmup 2 --no-cpu-baseline --no-batch --calibrate"
    out = [f"# Kernels of the transposition path, workload {workload} (MI355X, one GPU)", "",
           "Commands (from the repository root; cd /tmp && export TMPDIR=/tmp first):",
           f"  rocprofv3 --kernel-trace --stats -d <dir> -o trace -- {cmd}",
           f"  rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch -- {cmd}",
           f"  rocprofv3 --pmc WRITE_SIZE -d <dir> -o write -- {cmd}",
           f"  python -m paper_2501_06872_amd.profile_summary {workload} {passes} <dir>",
           "The run holds 2 warm-up + 5 timed steps and one 1 GiB device copy (--calibrate).", "",
           "Counter calibration (the 1 GiB copy: 1 GiB read, 1 GiB written):",
           f"  FETCH_SIZE read {cf:.0f} KiB -> factor {ffac:.3f};  WRITE_SIZE read {cw:.0f} KiB -> factor {wfac:.3f};"
           f"  copy {copy_us:.1f} us = {2 * (1 << 30) / copy_us / 1e3:.0f} GB/s",
           "HBM bytes per dispatch = factor x counter x 1024.", "",
           f"{'kernel':22s} {'calls':>5s} {'avg_us':>9s} {'total_ms':>9s} {'FETCH_KiB':>11s} {'WRITE_KiB':>11s} "
           f"{'HBM_GB/launch':>13s} {'GB/s':>7s}"]
    traffic = {}
    for k, (c, tot, full) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        f, w = agg["fetch"].get(k), agg["write"].get(k)
        if f is None or w is None:
            continue
        b = (ffac * f + wfac * w) * 1024
        traffic[k] = b
        avg = tot / c / 1000
        out.append(f"{k:22s} {c:5d} {avg:9.1f} {tot / 1e6:9.3f} {f:11.1f} {w:11.1f} {b / 1e9:13.3f} "
                   f"{b / (avg * 1e3):7.0f}")
    out += ["", "Kernel instances:"]
    seen = set()
    for k, (c, tot, full) in stats.items():
        if k.startswith("k_") and k not in seen:
            seen.add(k)
            out.append(f"  {k}: {full[:150]}")
    out += ["", "Machine-readable (bench.py reads these for roofline.traffic):",
            f"kernel_source_sha256={h.hexdigest()}"]
    for k, b in traffic.items():
        if k.startswith("k_"):
            out.append(f"traffic_bytes_per_launch {k}={b:.0f}")
    return "\n".join(out) + "\n"


def summarise_batch(d):
    """Kernel trace of bench.py --workload batch512: calls and durations per
    kernel over the whole run (plain per-graph launches, the batched plans
    over internal streams, the persistent kernel), and the persistent
    kernel's launches one by one (each transposes the whole batch)."""
    con = sqlite3.connect(os.path.join(d, "trace_results.db"))
    tr = con.execute("select name, duration from kernels").fetchall()
    stats = collections.OrderedDict()
    pers = []
    for n, dur in tr:
        k = label(n, 2)
        s = stats.setdefault(k, [0, 0.0])
        s[0] += 1
        s[1] += dur
        if k == "k_persistent":
            pers.append(dur / 1e6)
    cmd = "python3 bench.py --workload batch512 --steps 2 --warmup 1 --no-autotune"
    out = ["# Kernels of the 512-graph batch (MI355X, one GPU)", "",
           "Commands (from the repository root; cd /tmp && export TMPDIR=/tmp first):",
           f"  rocprofv3 --kernel-trace --stats -d <dir> -o trace -- {cmd}",
           "  python -m paper_2501_06872_amd.profile_summary batch512 --batch <dir>",
           "The run holds, per variant, 1 warm-up and 2 timed batches plus the launches that capture and check",
           "them: plain per-graph launches, batched plans over 8 internal streams (heuristic, learned), and the",
           "persistent kernel (heuristic, learned choices), one launch per batch.", "",
           f"{'kernel':22s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s}"]
    for k, (c, tot) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        out.append(f"{k:22s} {c:7d} {tot / c / 1000:10.1f} {tot / 1e6:10.3f}")
    if pers:
        out += ["", "k_persistent launches (ms, in launch order): " + ", ".join(f"{x:.3f}" for x in pers)]
    return "\n".join(out) + "\n"


def summarise_random_read(d, per, threads):
    """FETCH_SIZE of the random-access microbenchmark's HBM reads (each
    access a 4-byte word at a random place in an 8 GB array, so every one
    misses every cache): the calibrated bytes per access it implies, for the
    timed launches of `per` accesses per thread."""
    con = sqlite3.connect(os.path.join(d, "fetch_results.db"))
    rows = con.execute("select kernel_name, value from counters_collection where counter_name='FETCH_SIZE'").fetchall()
    per_disp = [v for k, v in rows if "k_random_global<0>" in k]  # reads of global memory
    copy = [v for k, v in rows if "copyBuffer" in k]
    accesses = threads * per
    timed = sorted(per_disp)[-3:]  # the three timed launches are the largest
    kib = sum(timed) / len(timed)
    out = ["# FETCH_SIZE of random 4-byte HBM reads (MI355X, one GPU)", "",
           "Commands (cd /tmp && export TMPDIR=/tmp PYTHONPATH=<repository root> first):",
           "  rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch -- python3 -m paper_2501_06872_amd.microbench "
           "--levels hbm --kinds read",
           f"  python -m paper_2501_06872_amd.profile_summary random-read --fetch <dir> {per} {threads}",
           f"({threads} threads x {per} accesses per thread in each timed launch; `per` from the run's JSON line)", "",
           f"FETCH_SIZE per timed launch: {kib:.0f} KiB for {accesses} accesses",
           f"  raw:                {kib * 1024 / accesses:.1f} bytes per access",
           f"  with the factor 2:  {2 * kib * 1024 / accesses:.1f} bytes per access"]
    if copy:
        out.append(f"(a device copy in the same run read {max(copy):.0f} KiB)")
    return "\n".join(out) + "\n"


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) == 5 and argv[1] == "--fetch":
        text = summarise_random_read(argv[2], int(argv[3]), int(argv[4]))
        with open(os.path.join(ROOT, "profiles", "gt_fetch_random_read.txt"), "w") as f:
            f.write(text)
        print(text)
        return
    if len(argv) == 3 and argv[1] == "--batch":
        text = summarise_batch(argv[2])
        path = os.path.join(ROOT, "profiles", f"gt_kernels_{argv[0]}.txt")
        with open(path, "w") as f:
            f.write(text)
        print(text)
        return
    if len(argv) != 3:
        raise SystemExit(__doc__)
    workload, passes, d = argv[0], int(argv[1]), argv[2]
    text = summarise(workload, passes, d)
    path = os.path.join(ROOT, "profiles", f"gt_kernels_{workload}.txt")
    with open(path, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
