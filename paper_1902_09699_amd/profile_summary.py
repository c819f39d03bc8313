"""Summarise a rocprofv3 SQLite output (rocpd) as a short text table:
per-kernel dispatch counts and mean durations, and, for counter runs, the
mean value per dispatch of each collected counter for each kernel.

    python -m paper_1902_09699_amd.profile_summary <dir-with-*results.db> [--top N]
"""
from __future__ import annotations

import argparse
import glob
import os
import sqlite3


def _db(path):
    if os.path.isdir(path):
        cands = sorted(glob.glob(os.path.join(path, "**", "*results.db"), recursive=True))
        if not cands:
            raise FileNotFoundError(f"no *results.db under {path}")
        path = cands[0]
    return sqlite3.connect(path)


def _short(name: str) -> str:
    """Kernel name without the library namespace (the FP32-reduction
    ablation build keeps its r32:: prefix)."""
    return name.replace("sip::", "").replace("r64::", "").replace("(anonymous namespace)::", "") \
        .replace("void ", "").split("(")[0]


def kernel_table(con, top=20):
    """top_kernels reports microseconds."""
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = [f"{'kernel':40s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>10s} {'pct':>6s}"]
    for name, calls, tot, avg, pct in rows[:top]:
        out.append(f"{_short(name)[:40]:40s} {calls:7d} {avg:9.2f} {tot / 1e3:10.3f} {pct:6.2f}")
    return "\n".join(out)


def kernel_grid_table(con, top=40):
    """Per kernel and launch shape (grid and work-group size): dispatch
    count and mean duration, so launches of different workloads in one
    process (a batch, a single grid, a served mix) are told apart."""
    q = ("select name, grid_x, workgroup_x, count(*), avg(duration), sum(duration) from kernels "
         "group by 1, 2, 3 order by 6 desc")
    rows = con.execute(q).fetchall()
    out = [f"{'kernel':40s} {'grid_x':>9s} {'wg':>5s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>10s}"]
    for name, gx, wx, calls, avg, tot in rows[:top]:
        out.append(f"{_short(name)[:40]:40s} {gx:9d} {wx:5d} {calls:7d} {avg / 1e3:9.2f} {tot / 1e6:10.3f}")
    return "\n".join(out)


def counter_table(con):
    try:
        cols = [c[1] for c in con.execute("pragma table_info(counters_collection)")]
        if not cols or not con.execute("select count(*) from counters_collection").fetchone()[0]:
            return ""
    except sqlite3.Error:
        return ""
    kcol = "kernel_name" if "kernel_name" in cols else "name"
    vcol = "value" if "value" in cols else "counter_value"
    q = (f"select {kcol}, counter_name, avg({vcol}), count(*) from counters_collection "
         f"group by 1, 2 order by 1, 2")
    out = [f"{'kernel':40s} {'counter':12s} {'mean/dispatch':>16s} {'dispatches':>10s}"]
    for name, cname, val, n in con.execute(q):
        out.append(f"{_short(name)[:40]:40s} {cname:12s} {val:16.1f} {n:10d}")
    return "\n".join(out)


def counter_means(con, counter):
    """{short kernel name: mean counter value per dispatch}."""
    cols = [c[1] for c in con.execute("pragma table_info(counters_collection)")]
    kcol = "kernel_name" if "kernel_name" in cols else "name"
    vcol = "value" if "value" in cols else "counter_value"
    q = f"select {kcol}, avg({vcol}) from counters_collection where counter_name = ? group by 1"
    return {_short(n): v for n, v in con.execute(q, (counter,))}


def traffic(fetch_path, write_path, kernel, copy_bytes):
    """HBM bytes per launch of `kernel` from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for the plain copy kernel k_copy that reads and writes copy_bytes."""
    f = counter_means(_db(fetch_path), "FETCH_SIZE")
    w = counter_means(_db(write_path), "WRITE_SIZE")
    kf = next(v for k, v in f.items() if k.startswith(kernel))
    kw = next(v for k, v in w.items() if k.startswith(kernel))
    cf = f["k_copy"] * 1024.0 / copy_bytes
    cw = w["k_copy"] * 1024.0 / copy_bytes
    read = kf * 1024.0 / cf
    written = kw * 1024.0 / cw
    return {"kernel": kernel, "fetch_kib": kf, "write_kib": kw, "copy_fetch_factor": cf,
            "copy_write_factor": cw, "hbm_bytes_read": read, "hbm_bytes_written": written,
            "hbm_bytes_per_launch": read + written}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("path")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--write-db", help="with --kernel: traffic from a FETCH_SIZE db (path) and this WRITE_SIZE db")
    ap.add_argument("--kernel")
    ap.add_argument("--copy-bytes", type=float, default=256 * (1 << 20))
    ap.add_argument("--by-grid", action="store_true", help="kernel trace per launch shape")
    a = ap.parse_args()
    if a.write_db:
        import json
        print(json.dumps(traffic(a.path, a.write_db, a.kernel, a.copy_bytes), indent=1))
        return
    con = _db(a.path)
    if a.by_grid:
        print(kernel_grid_table(con, a.top))
        return
    ct = counter_table(con)
    print(ct if ct else kernel_table(con, a.top))


if __name__ == "__main__":
    main()
