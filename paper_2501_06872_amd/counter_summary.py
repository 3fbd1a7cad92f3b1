"""Summarise rocprofv3 counter runs of bench.py into profiles/gt_counters_<workload>.txt.

    python -m paper_2501_06872_amd.counter_summary <workload> <passes> <dir> <edges>

<dir> holds three rocprofv3 --pmc databases of one workload (sq1_results.db,
sq2_results.db, sq3_results.db), made by the commands the summary prints.
Per kernel and dispatch (averaged over the dispatches of the run) it lists
the shader-sequencer counters (wave cycles, waits, LDS and memory
instructions, LDS bank conflicts) and the L2 atomic and write-request
counts, with the ratios read from them:

  waiting     SQ_WAIT_ANY / SQ_WAVE_CYCLES: share of wave time spent waiting
              (on memory, LDS or a barrier)
  lds_active  SQ_LDS_IDX_ACTIVE / (SQ_BUSY_CYCLES x 8): share of the kernel's
              cycles in which a compute unit's LDS pipeline works
              (SQ_BUSY_CYCLES sums the 32 shader engines of 8 compute units)
  bank_confl  SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: share of those LDS
              cycles lost to bank conflicts
  valu_busy   SQ_INSTS_VALU / (SQ_BUSY_CYCLES x 8): wave64 VALU instructions
              per compute-unit cycle (4 SIMDs, 4 cycles per wave64 VALU
              instruction: 1.0 is the issue limit)
  lds/tile-wave, valu/edge: LDS wave instructions per 64 edges, VALU wave
              instructions per edge
"""
import collections
import os
import sqlite3
import sys

from paper_2501_06872_amd.profile_summary import label

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PASSES = {
    "sq1": ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS",
            "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_LDS"],
    "sq2": ["SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_ADDR_CONFLICT", "SQ_LDS_IDX_ACTIVE",
            "SQ_INSTS_LDS_ATOMIC", "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"],
    "sq3": ["SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_INST_LEVEL_VMEM",
            "SQ_INSTS_SALU", "SQ_INSTS_SMEM", "SQ_LEVEL_WAVES", "SQ_CYCLES",
            "TCC_ATOMIC", "TCC_EA0_WRREQ", "TCC_EA0_WRREQ_64B", "TCC_EA0_RDREQ"],
}
KERNELS = ("k_hist", "k_lsd_pass0", "k_tile_hist", "k_lsd_pass1", "k_lsd_pass2", "k_big_count", "k_big_scan",
           "k_final", "k_hlh_count", "k_hlh_scatter")


def command(workload, tag):
    return (f"rocprofv3 --pmc {' '.join(PASSES[tag])} -d <dir> -o {tag} -- "
            f"python3 bench.py --workload {workload} --steps 2 --warmup 1 --no-cpu-baseline --no-batch")


def summarise(workload, passes, d, edges):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for tag in PASSES:
        con = sqlite3.connect(os.path.join(d, f"{tag}_results.db"))
        rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
        per = collections.defaultdict(float)  # (dispatch, kernel, counter) summed over dimensions
        for disp, k, c, v in rows:
            per[(disp, label(k, passes), c)] += v
        for (disp, k, c), v in per.items():
            vals[k][c].append(v)
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}
    out = [f"# Shader and L2 counters of the transposition kernels, workload {workload} (MI355X, one GPU)", "",
           "Commands (from the repository root; cd /tmp && export TMPDIR=/tmp first):"]
    out += [f"  {command(workload, tag)}" for tag in PASSES]
    out += [f"  python -m paper_2501_06872_amd.counter_summary {workload} {passes} <dir> {edges}",
            "Values: per dispatch, averaged over the dispatches of the run (3 transpositions).", ""]
    hdr = (f"{'kernel':14s} {'waiting':>8s} {'lds_active':>10s} {'bank_confl':>10s} {'valu_busy':>9s} "
           f"{'lds/64e':>8s} {'valu/edge':>9s} {'atomics':>12s} {'wrreq':>12s} {'wrreq64B':>12s}")
    out.append(hdr)
    for k in KERNELS:
        a = avg.get(k)
        if not a:
            continue
        g = lambda c: a.get(c, float("nan"))
        waiting = g("SQ_WAIT_ANY") / g("SQ_WAVE_CYCLES")
        lds_active = g("SQ_LDS_IDX_ACTIVE") / (8 * g("SQ_BUSY_CYCLES"))
        bank = g("SQ_LDS_BANK_CONFLICT") / g("SQ_LDS_IDX_ACTIVE")
        valu = g("SQ_INSTS_VALU") / (8 * g("SQ_BUSY_CYCLES"))
        lpe = g("SQ_INSTS_LDS") * 64 / edges
        vpe = g("SQ_INSTS_VALU") / edges
        out.append(f"{k:14s} {waiting:8.3f} {lds_active:10.3f} {bank:10.3f} {valu:9.3f} {lpe:8.2f} {vpe:9.3f} "
                   f"{g('TCC_ATOMIC'):12.0f} {g('TCC_EA0_WRREQ'):12.0f} {g('TCC_EA0_WRREQ_64B'):12.0f}")
    out += ["", "Raw counters (per dispatch):"]
    for k in KERNELS:
        a = avg.get(k)
        if not a:
            continue
        out.append(f"  {k}:")
        for c in sorted(a):
            out.append(f"    {c:26s} {a[c]:.6g}")
    return "\n".join(out) + "\n"


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 4:
        raise SystemExit(__doc__ + "\n(arguments: <workload> <passes> <dir> <edges>)")
    workload, passes, d, edges = argv[0], int(argv[1]), argv[2], int(argv[3])
    text = summarise(workload, passes, d, edges)
    with open(os.path.join(ROOT, "profiles", f"gt_counters_{workload}.txt"), "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
