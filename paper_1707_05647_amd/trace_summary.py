"""Per-kernel launch durations from a rocprofv3 kernel trace, split by how
the launch ran.

    python -m paper_1707_05647_amd.trace_summary KERNEL_TRACE_CSV [--only TEXT ...]

Reads the ``kernel_trace.csv`` of a ``rocprofv3 --kernel-trace`` run and
prints, per library kernel and launch shape (grid and workgroup size), the
launches that ran alone and those that overlapped another library launch
(count, mean, median, extremes).  The benchmark's lanes run one lane's star
pass beside the other lane's build or star pass, so those launches share the
compute units and take longer each.  The benchmark's
one-lane and lanes' HIP-event averages are to be compared with the "alone"
and "overlapped" rows of the timed launch shape.  With ``--only``, the table
lists only the launches whose full kernel name (template arguments included)
contains one of the given texts; overlap is still judged against every
library launch.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict

from paper_1707_05647_amd.traffic import short_name


def _int(row, *keys):
    for k in keys:
        if k in row and row[k] != "":
            return int(float(row[k]))
    return 0


def load(path):
    out = []
    with open(path) as f:
        for row in csv.DictReader(f):
            short = short_name(row.get("Kernel_Name", ""))
            if short is None:
                continue
            grid = _int(row, "Grid_Size_X", "Grid_Size")
            wg = _int(row, "Workgroup_Size_X", "Workgroup_Size")
            out.append((short, int(row["Start_Timestamp"]), int(row["End_Timestamp"]), grid, wg,
                        _int(row, "Queue_Id"), row.get("Kernel_Name", "")))
    return out


def overlapped(launches):
    """Per launch (start-sorted), whether it overlaps another one in time."""
    order = sorted(range(len(launches)), key=lambda i: launches[i][1])
    flag = [False] * len(launches)
    end_max, end_idx = -1, -1
    for i in order:
        s, e = launches[i][1], launches[i][2]
        if s < end_max:
            flag[i] = True
            flag[end_idx] = True
        if e > end_max:
            end_max, end_idx = e, i
    return flag


def summarize(rows, only=None):
    """The table; `only`: texts, one of which a listed launch's full kernel
    name contains (None: every launch)."""
    ov_all = overlapped(rows)
    by_kernel = defaultdict(list)
    for r, o in zip(rows, ov_all):
        if only and not any(t in r[6] for t in only):
            continue
        by_kernel[r[0]].append((r, o))
    lines = ["| Kernel | grid x workgroup | launches | ran | avg ms | median ms | min ms | max ms |",
             "|:--|--:|--:|:--|--:|--:|--:|--:|"]
    for k in sorted(by_kernel, key=lambda k: -sum(r[2] - r[1] for r, _ in by_kernel[k])):
        groups = defaultdict(list)
        for r, o in by_kernel[k]:
            groups[(r[3], r[4], o)].append((r[2] - r[1]) / 1e6)
        for (grid, wg, o), d in sorted(groups.items(), key=lambda kv: (-len(kv[1]), kv[0])):
            d.sort()
            med = d[len(d) // 2] if len(d) % 2 else 0.5 * (d[len(d) // 2 - 1] + d[len(d) // 2])
            lines.append(f"| {k} | {grid // max(wg, 1)} x {wg} | {len(d)} | "
                         f"{'overlapped' if o else 'alone'} | {sum(d) / len(d):.3f} | "
                         f"{med:.3f} | {d[0]:.3f} | {d[-1]:.3f} |")
    return "\n".join(lines)


if __name__ == "__main__":
    args = sys.argv[1:]
    only = None
    if "--only" in args:
        i = args.index("--only")
        only, args = args[i + 1:], args[:i]
    if len(args) != 1 or (only is not None and not only):
        raise SystemExit(__doc__)
    print(summarize(load(args[0]), only))
