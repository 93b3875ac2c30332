"""Summarise rocprofv3 CSV output per kernel and launch size.

    python -m paper_2204_13304_amd.profile_summary <rocprofv3 output dir>
    python -m paper_2204_13304_amd.profile_summary <dir> --iteration KERNEL K

Reads the rocpd SQLite database rocprofv3 writes by default (*.db), or
its CSV output (--output-format csv), and prints: the per-kernel
statistics (--stats); per (kernel name, grid size, workgroup size) the
number of launches and the average / total duration (--kernel-trace);
and per (kernel, grid size, counter) the mean value per dispatch (--pmc).
With --iteration it lists instead, in launch order, the kernels of a trace
database that ran after the (K-1)-th launch of a kernel whose name contains
KERNEL, up to and including its K-th launch (one solver iteration when
KERNEL is the iteration's last kernel), with their durations.
Only the standard library is used.
"""
from __future__ import annotations

import csv
import glob
import os
import re
import sqlite3
import sys
from collections import defaultdict


def _short(name: str, width: int = 90) -> str:
    name = re.sub(r"\s+", " ", name)
    return name if len(name) <= width else name[: width - 3] + "..."


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    return None


def trace_table(path: str) -> str:
    groups = defaultdict(list)
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = _col(row, "Kernel_Name", "KernelName", "Name")
            start = _col(row, "Start_Timestamp", "BeginNs", "Start")
            end = _col(row, "End_Timestamp", "EndNs", "End")
            grid = _col(row, "Grid_Size", "Grid_Size_X", "Grid", "grd")
            wg = _col(row, "Workgroup_Size", "Workgroup_Size_X", "wgr")
            if name is None or start is None or end is None:
                continue
            groups[(name, grid, wg)].append((int(end) - int(start)) / 1e3)
    lines = ["kernel | grid | workgroup | launches | avg_us | total_ms"]
    for (name, grid, wg), d in sorted(groups.items(),
                                      key=lambda kv: -sum(kv[1])):
        lines.append(f"{_short(name)} | {grid} | {wg} | {len(d)} | "
                     f"{sum(d) / len(d):.2f} | {sum(d) / 1e3:.3f}")
    return "\n".join(lines)


def stats_table(path: str) -> str:
    out = []
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = _col(row, "Name", "KernelName", "Kernel_Name")
            calls = _col(row, "Calls", "calls")
            avg = _col(row, "AverageNs", "Average_ns", "AvgNs")
            tot = _col(row, "TotalDurationNs", "Total_ns", "TotalNs")
            pct = _col(row, "Percentage", "percentage")
            out.append(f"{_short(name)} | calls {calls} | avg_ns {avg} | "
                       f"total_ns {tot} | {pct}%")
    return "\n".join(out)


def counter_table(path: str) -> str:
    per = defaultdict(lambda: defaultdict(list))
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = _col(row, "Kernel_Name", "KernelName", "Name")
            cname = _col(row, "Counter_Name", "CounterName")
            val = _col(row, "Counter_Value", "CounterValue", "Value")
            grid = _col(row, "Grid_Size", "Grid")
            if name is None or cname is None or val is None:
                continue
            per[(name, grid)][cname].append(float(val))
    lines = ["kernel | grid | counter | dispatches | mean per dispatch"]
    for (name, grid), cs in per.items():
        for c, v in cs.items():
            lines.append(f"{_short(name)} | {grid} | {c} | {len(v)} | "
                         f"{sum(v) / len(v):.1f}")
    return "\n".join(lines)


def db_tables(path: str) -> str:
    con = sqlite3.connect(path)
    out = ["### per kernel (all launches)",
           "kernel | calls | avg_us | total_ms | percent"]
    for name, calls, tot, avg, pct in con.execute(
            "select name, total_calls, total_duration, average, percentage "
            "from top_kernels order by total_duration desc"):
        # top_kernels reports microseconds
        out.append(f"{_short(name)} | {calls} | {avg:.2f} | "
                   f"{tot / 1e3:.3f} | {pct:.1f}")
    rows = con.execute(
        "select name, grid_x, grid_y, grid_z, workgroup_x, count(*), "
        "avg(duration), sum(duration) from kernels "
        "group by name, grid_x, grid_y, grid_z, workgroup_x "
        "order by sum(duration) desc").fetchall()
    if rows:
        out += ["", "### per kernel and launch size",
                "kernel | grid | workgroup | launches | avg_us | total_ms"]
        for name, gx, gy, gz, wx, cnt, avg, tot in rows:
            out.append(f"{_short(name)} | {gx}x{gy}x{gz} | {wx} | {cnt} | "
                       f"{avg / 1e3:.2f} | {tot / 1e6:.3f}")
    rows = con.execute(
        "select kernel_name, grid_size, counter_name, count(*), avg(value) "
        "from counters_collection group by kernel_name, grid_size, "
        "counter_name order by kernel_name, grid_size").fetchall()
    if rows:
        out += ["", "### PMC counters (mean per dispatch)",
                "kernel | grid | counter | dispatches | mean"]
        for name, grid, cname, cnt, val in rows:
            out.append(f"{_short(name)} | {grid} | {cname} | {cnt} | "
                       f"{val:.1f}")
    con.close()
    return "\n".join(out)


def iteration_table(path: str, kernel: str, k: int) -> str:
    con = sqlite3.connect(path)
    rows = con.execute("select name, grid_x, start, end, duration from "
                       "kernels order by start").fetchall()
    con.close()
    ends = [i for i, r in enumerate(rows) if kernel in r[0]]
    if k < 1 or k > len(ends):
        return f"{len(ends)} launches of {kernel}: no iteration {k}"
    a = ends[k - 2] + 1 if k > 1 else 0
    b = ends[k - 1]
    out = [f"### launches {a} .. {b} (iteration {k} of {len(ends)}): "
           f"sum {sum(r[4] for r in rows[a:b + 1]) / 1e3:.1f} us, "
           f"first start to last end {(rows[b][3] - rows[a][2]) / 1e3:.1f} us",
           "kernel | grid | us"]
    for name, gx, _, _, dur in rows[a:b + 1]:
        out.append(f"{_short(name)} | {gx} | {dur / 1e3:.1f}")
    return "\n".join(out)


def main(argv):
    if len(argv) == 5 and argv[2] == "--iteration":
        for p in sorted(glob.glob(os.path.join(argv[1], "**", "*.db"),
                                  recursive=True)):
            print(f"## {os.path.relpath(p, argv[1])}")
            print(iteration_table(p, argv[3], int(argv[4])))
        return 0
    if len(argv) != 2:
        print(__doc__)
        return 2
    root = argv[1]
    for pattern, fn, title in (
            ("*kernel_stats.csv", stats_table, "rocprofv3 --stats"),
            ("*kernel_trace.csv", trace_table, "per kernel and launch size"),
            ("*counter_collection.csv", counter_table, "PMC counters"),
            ("*.db", db_tables, "rocpd database")):
        for p in sorted(glob.glob(os.path.join(root, "**", pattern),
                                  recursive=True)):
            print(f"## {title}: {os.path.relpath(p, root)}")
            print(fn(p))
            print()
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
