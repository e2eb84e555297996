"""Summarise a rocprofv3 kernel trace (CSV) per kernel and launch shape.

    python -m paper_2507_23612_amd.tracesum <dir-with-*_kernel_trace.csv> [top]

Prints, per (kernel, grid, workgroup) group: launches, total, average, min
and max duration in ms, sorted by total time.  Grouping by launch shape
separates, e.g., the full-block stencil launches from the single-vector
launches of the Lanczos bound.
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import sys


def summarise(path, top=15):
    files = glob.glob(os.path.join(path, "*_kernel_trace.csv")) if os.path.isdir(path) else [path]
    if not files:
        raise FileNotFoundError(f"no *_kernel_trace.csv under {path}")
    groups = collections.defaultdict(list)
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"]
                short = name.split("(")[0].replace("void ", "")
                key = (short, f"grid={r['Grid_Size_X']}x{r['Grid_Size_Y']}x{r['Grid_Size_Z']}",
                       f"wg={r['Workgroup_Size_X']}x{r['Workgroup_Size_Y']}")
                groups[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    total = sum(sum(v) for v in groups.values())
    out = ["| kernel | launch | calls | total ms | avg ms | min ms | max ms | % |",
           "|---|---|---|---|---|---|---|---|"]
    for (k, g, w), v in rows[:top]:
        out.append(f"| `{k}` | {g} {w} | {len(v)} | {sum(v):.3f} | {sum(v) / len(v):.4f} | {min(v):.4f} | "
                   f"{max(v):.4f} | {100 * sum(v) / total:.1f} |")
    return "\n".join(out)


def counters(path, kernel_sub, counter):
    """Per-dispatch values of `counter` for kernels whose name contains
    `kernel_sub`, grouped by grid shape: {grid: [values]}."""
    files = glob.glob(os.path.join(path, "*_counter_collection.csv")) if os.path.isdir(path) else [path]
    out = collections.defaultdict(list)
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if kernel_sub in r["Kernel_Name"] and r["Counter_Name"] == counter:
                    g = f"{r.get('Grid_Size', '')}"
                    out[g].append(float(r["Counter_Value"]))
    return out


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--counter":
        # --counter <dir> <kernel substring> <counter name>
        for g, v in counters(sys.argv[2], sys.argv[3], sys.argv[4]).items():
            print(f"{sys.argv[3]} grid={g} {sys.argv[4]}: n={len(v)} avg={sum(v) / len(v):.1f} min={min(v):.1f} "
                  f"max={max(v):.1f}")
    else:
        print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 15))
