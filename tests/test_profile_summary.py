"""The rocprofv3 summary on the host: counter calibration against the 1 GiB
copy and the per-launch byte figures bench.py reads back."""
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

LSD0 = "void gt::k_lsd<8, 16, 8, true, false, false, true, unsigned int>(gt::LsdArgs)"
LSD1 = "void gt::k_lsd<8, 16, 9, false, false, true, true, unsigned int>(gt::LsdArgs)"
COPY = "__amd_rocclr_copyBuffer"


def make_dbs(d):
    con = sqlite3.connect(os.path.join(d, "trace_results.db"))
    con.execute("create table kernels (dispatch_id, name, duration)")
    rows = [(1, COPY, 400_000), (2, LSD0, 4_000_000), (3, LSD0, 6_000_000), (4, LSD1, 5_000_000)]
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    for tag, cn, copy_kib, lsd0, lsd1 in (("fetch", "FETCH_SIZE", 1 << 19, 1000.0, 3000.0),
                                          ("write", "WRITE_SIZE", 1 << 20, 2000.0, 500.0)):
        con = sqlite3.connect(os.path.join(d, f"{tag}_results.db"))
        con.execute("create table counters_collection (kernel_name, counter_name, value, grid_size)")
        con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                        [(COPY, cn, copy_kib, 1), (LSD0, cn, lsd0, 1), (LSD0, cn, lsd0, 1), (LSD1, cn, lsd1, 1)])
        con.commit()


def test_summary_scales_counters_by_the_copy(tmp_path):
    from paper_2501_06872_amd import profile_summary as ps
    make_dbs(str(tmp_path))
    text = ps.summarise("toy", 2, str(tmp_path))
    # FETCH reads half of the copy's bytes (factor 2), WRITE all of them (factor 1)
    assert "factor 2.000" in text and "factor 1.000" in text
    lines = dict(l.split(" ", 1)[1].split("=") for l in text.splitlines() if l.startswith("traffic_bytes_per_launch"))
    assert int(lines["k_lsd_pass0"]) == (2 * 1000 + 2000) * 1024
    assert int(lines["k_lsd_pass1"]) == (2 * 3000 + 500) * 1024
    # two launches of pass 0 averaging 5 ms
    row = [l for l in text.splitlines() if l.startswith("k_lsd_pass0 ")][0].split()
    assert row[1] == "2" and float(row[2]) == 5000.0
    assert "kernel_source_sha256=" in text
