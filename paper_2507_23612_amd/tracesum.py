"""Summarise a rocprofv3 kernel trace (CSV) per kernel and launch shape.

    python -m paper_2507_23612_amd.tracesum <dir-with-*_kernel_trace.csv> [top]
    python -m paper_2507_23612_amd.tracesum --counter <dir> <kernel substring> <counter>
    python -m paper_2507_23612_amd.tracesum --record <trace dir> <FETCH_SIZE dir> <WRITE_SIZE dir> \
        <kernel substring> <tile> <title> <command file> [source files, comma-separated] [counter dir]

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


def kernel_source_digest(sources=("stencil.hip",)):
    """sha256 of a kernel's source files: a counter record applies only to
    the kernel code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _largest_grid(vals):
    """The group with the largest grid (the full-block launches)."""
    g = max(vals, key=lambda k: int(k) if k.isdigit() else -1)
    return g, vals[g]


def _avg_ms_largest_grid(trace_dir, kernel_sub):
    files = glob.glob(os.path.join(trace_dir, "*_kernel_trace.csv"))
    groups = collections.defaultdict(list)
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if kernel_sub in r["Kernel_Name"]:
                    g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                    groups[g].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    g = max(groups)
    return g, groups[g]


def _calibration(path, counter):
    """Counter value (KiB) of the 1 GiB device copy that `bench.py
    --calib-copy` issues before any other large copy (the first copy
    dispatch above 64 MiB), and the factor that maps it to 1 GiB."""
    rows = []
    for f in glob.glob(os.path.join(path, "*_counter_collection.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    rows.sort()
    first = next(v for _, v in rows if v > 65536.0)
    return first, 1048576.0 / first


def sq_lines(sq_dir, kernel_sub, avg_ms):
    """Per-launch averages of the instruction-counter pass (full-block
    launches) and the matrix-core busy fraction derived from them.
    GRBM_GUI_ACTIVE is summed over the 8 XCDs, so one XCD's active cycles
    are a eighth of it; SQ_VALU_MFMA_BUSY_CYCLES is summed over the 1024
    SIMDs (256 CUs x 4)."""
    names = set()
    for f in glob.glob(os.path.join(sq_dir, "*_counter_collection.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if kernel_sub in r["Kernel_Name"]:
                    names.add(r["Counter_Name"])
    vals = {}
    for n in sorted(names):
        _, v = _largest_grid(counters(sq_dir, kernel_sub, n))
        vals[n] = sum(v) / len(v)
    out = ["", "## Instruction counters (full-block launches, per launch)", ""]
    out += [f"- {n}: {v:.4g}" for n, v in vals.items()]
    if "GRBM_GUI_ACTIVE" in vals and "SQ_VALU_MFMA_BUSY_CYCLES" in vals:
        gui = vals["GRBM_GUI_ACTIVE"] / 8.0
        busy = vals["SQ_VALU_MFMA_BUSY_CYCLES"] / (gui * 1024.0)
        out += [f"- GPU active per XCD: {gui:.0f} cycles ({gui / 2.4e6:.4f} ms at 2.4 GHz; "
                f"trace average {avg_ms:.4f} ms)",
                f"- matrix-core busy fraction: SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x 1024 SIMDs) = {busy:.3f}"]
    if "SQ_WAVE_CYCLES" in vals and "SQ_WAIT_INST_ANY" in vals and vals["SQ_WAVE_CYCLES"] > 0:
        out.append(f"- waves waiting on any instruction dependency: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES = "
                   f"{vals['SQ_WAIT_INST_ANY'] / vals['SQ_WAVE_CYCLES']:.3f}")
    return out


def record(trace_dir, fetch_dir, write_dir, kernel_sub, tile, title, cmds, digest, sq_dir=None):
    """Markdown summary of one kernel: trace statistics, per-launch
    FETCH_SIZE / WRITE_SIZE scaled by the copy calibration, optionally the
    instruction-counter pass, and the record lines bench.py reads (traffic
    per launch, tile, source digest)."""
    grid, durs = _avg_ms_largest_grid(trace_dir, kernel_sub)
    fg, fv = _largest_grid(counters(fetch_dir, kernel_sub, "FETCH_SIZE"))
    wg, wv = _largest_grid(counters(write_dir, kernel_sub, "WRITE_SIZE"))
    fetch = sum(fv) / len(fv)
    write = sum(wv) / len(wv)
    cf_raw, cf = _calibration(fetch_dir, "FETCH_SIZE")
    cw_raw, cw = _calibration(write_dir, "WRITE_SIZE")
    traffic = (fetch * cf + write * cw) * 1024.0
    out = [f"# {title}", "", "Commands (from the repository root on the MI355X box):", "", "```"]
    out += cmds
    out += ["```", "", "## Kernel trace (grouped by kernel and launch shape)", "", summarise(trace_dir, 20), "",
            f"## `{kernel_sub}` full-block launches (grid {grid} work-items)", "",
            f"- launches: {len(durs)}, average {sum(durs) / len(durs):.4f} ms, min {min(durs):.4f}, "
            f"max {max(durs):.4f}",
            f"- FETCH_SIZE per launch: {fetch:.1f} KiB raw over {len(fv)} dispatches (grid {fg})",
            f"- WRITE_SIZE per launch: {write:.1f} KiB raw over {len(wv)} dispatches (grid {wg})",
            f"- calibration (1 GiB device copy): FETCH_SIZE reads {cf_raw:.1f} KiB -> factor {cf:.3f}; "
            f"WRITE_SIZE reads {cw_raw:.1f} KiB -> factor {cw:.3f}",
            f"- HBM traffic per launch: {fetch * cf / 1024:.1f} MiB fetched + {write * cw / 1024:.1f} MiB written "
            f"= {traffic / 2**20:.1f} MiB"]
    if sq_dir:
        out += sq_lines(sq_dir, kernel_sub, sum(durs) / len(durs))
    out += ["", "Record read by bench.py (applies while the kernel sources hash to the digest):", "",
            f"- record kernel: {kernel_sub}",
            f"- record tile: {tile}",
            f"- record traffic_bytes_per_launch: {traffic:.0f}",
            f"- record avg_launch_ms: {sum(durs) / len(durs):.5f}",
            f"- record source_sha256: {digest}", ""]
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--record":
        with open(sys.argv[8]) as fh:
            cmds = [ln.rstrip("\n") for ln in fh if ln.strip()]
        srcs = tuple(sys.argv[9].split(",")) if len(sys.argv) > 9 else ("stencil.hip",)
        sq = sys.argv[10] if len(sys.argv) > 10 else None
        print(record(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], sys.argv[7], cmds,
                     kernel_source_digest(srcs), sq))
        sys.exit(0)
    if len(sys.argv) > 2 and sys.argv[1] == "--counter":
        # --counter <dir> <kernel substring> <counter name>
        for g, v in counters(sys.argv[2], sys.argv[3], sys.argv[4]).items():
            print(f"{sys.argv[3]} grid={g} {sys.argv[4]}: n={len(v)} avg={sum(v) / len(v):.1f} min={min(v):.1f} "
                  f"max={max(v):.1f}")
    else:
        print(summarise(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 15))
