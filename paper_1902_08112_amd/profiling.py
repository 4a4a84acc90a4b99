"""Summaries of rocprofv3 output: per-kernel durations and HBM traffic.

    python -m paper_1902_08112_amd.profiling stats --trace <kernel_trace.csv> --out <summary.md>
        --command "<the profiled command>" [--kernel NAME] [--grid N] [--top 25]
    python -m paper_1902_08112_amd.profiling traffic --fetch <counter_collection.csv>
        --write <counter_collection.csv> --kernel NAME --grid N --copy-bytes B --algorithmic-bytes A
        --workload W --out <traffic.json> --command "<...>" --sources f1 f2 ...
    python -m paper_1902_08112_amd.profiling counters --csv <counter_collection.csv> --kernel NAME
        [--kernel NAME ...] [--grid N] --out <summary.md> --command "<...>"

stats: duration statistics per kernel (and, for one kernel at one grid size,
the per-dispatch mean that the bench's live HIP-event measurement is compared
with) from a --kernel-trace CSV.

traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of one kernel at one
grid size, each scaled by what the same counter reads for the plain device
copy of copy_bytes that bench.py runs after its timed region (the counters
cover part of the memory channels; the copy's known size calibrates them).
The record carries a hash of the kernel's source files: bench.py reports the
traffic only while the sources are unchanged.

counters: the mean per dispatch of every counter of a --pmc pass for each named
kernel (at its largest grid, the finest level, or the one asked for), with the
per-wave ratios of the SQ counters when they are present: instructions per wave,
and the fractions of the waves' lifetime (SQ_WAVE_CYCLES) spent issuing VALU,
waiting on any instruction and waiting on LDS.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def sources_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(p.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def short(name):
    n = name.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*", "", n).replace("void ", "").replace("pff::", "")
    return n.strip()


def _col(row, *cands):
    for c in cands:
        if c in row:
            return row[c]
    raise KeyError(cands)


def _grid(row):
    for c in ("Grid_Size", "Grid_Size_X", "Grid_X"):
        if c in row:
            g = int(float(row[c]))
            for e in ("Grid_Size_Y", "Grid_Y"), ("Grid_Size_Z", "Grid_Z"):
                for cc in e:
                    if cc in row:
                        g *= max(1, int(float(row[cc])))
            return g
    return -1


def trace_rows(path):
    with open(path) as f:
        for r in csv.DictReader(f):
            t0 = int(_col(r, "Start_Timestamp", "start"))
            t1 = int(_col(r, "End_Timestamp", "end"))
            yield short(_col(r, "Kernel_Name", "Name", "name")), _grid(r), (t1 - t0) * 1e-9


def stats(a):
    per = {}
    per_grid = {}
    for name, grid, dt in trace_rows(a.trace):
        per.setdefault(name, []).append(dt)
        per_grid.setdefault((name, grid), []).append(dt)
    total = sum(sum(v) for v in per.values())
    lines = [f"# Kernel durations: {os.path.basename(a.out)}", "",
             "Command (from the repository root on the GPU box):", "", "```", a.command, "```", "",
             f"Kernel dispatches: {sum(len(v) for v in per.values())}, total kernel time {total * 1e3:.3f} ms.", ""]
    for k, kname in enumerate(a.kernel or []):
        # the finest level's launches: the largest grid of that kernel (or the one asked for)
        grids = [g for (n, g) in per_grid if n == kname]
        if not grids:
            continue
        g = a.grid if a.grid is not None else max(grids)
        v = per_grid.get((kname, g), [])
        if v:
            lines += [f"{'Dominant kernel' if k == 0 else 'Kernel'} `{kname}` at grid {g}: {len(v)} dispatches, "
                      f"mean {statistics.mean(v) * 1e6:.2f} us, median {statistics.median(v) * 1e6:.2f} us, "
                      f"min {min(v) * 1e6:.2f} us, max {max(v) * 1e6:.2f} us.", ""]
    lines += ["| kernel | calls | total ms | mean us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:a.top]:
        lines.append(f"| `{name}` | {len(v)} | {sum(v) * 1e3:.3f} | {statistics.mean(v) * 1e6:.2f} | "
                     f"{min(v) * 1e6:.2f} | {max(v) * 1e6:.2f} | {100 * sum(v) / total:.1f} |")
    lines += ["", "Per kernel and grid (the grid is the launch's total work-item count; one grid is one level):", "",
              "| kernel | grid | calls | total ms | mean us | % |", "|---|---:|---:|---:|---:|---:|"]
    for (name, g), v in sorted(per_grid.items(), key=lambda kv: -sum(kv[1]))[:a.top]:
        lines.append(f"| `{name}` | {g} | {len(v)} | {sum(v) * 1e3:.3f} | {statistics.mean(v) * 1e6:.2f} | "
                     f"{100 * sum(v) / total:.1f} |")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counter_values(path, counter, kernel, grid):
    vals = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if _col(r, "Counter_Name") != counter:
                continue
            if not re.search(kernel, short(_col(r, "Kernel_Name"))):
                continue
            if grid is not None and _grid(r) != grid:
                continue
            vals.append(float(_col(r, "Counter_Value")))
    return vals


def largest_grid(path, kernel):
    """The largest grid at which a kernel (regex on the short name) was dispatched in a counter CSV."""
    grids = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if re.search(kernel, short(_col(r, "Kernel_Name"))):
                grids.append(_grid(r))
    return max(grids) if grids else None


def traffic(a):
    kern = "^" + re.escape(a.kernel) + "$"
    # without a grid: the kernel's finest level, and the largest copy (one fine-level vector)
    grid = a.grid if a.grid is not None else largest_grid(a.fetch, kern)
    copy_grid = a.copy_grid if a.copy_grid is not None else largest_grid(a.fetch, a.copy_kernel)
    out = {"workload": a.workload, "kernel": a.kernel, "grid": grid, "command": a.command,
           "sources": a.sources, "sources_sha": sources_sha(a.sources)}
    tot = 0.0
    for counter, path in (("FETCH_SIZE", a.fetch), ("WRITE_SIZE", a.write)):
        k = counter_values(path, counter, kern, grid)
        c = counter_values(path, counter, a.copy_kernel, copy_grid)
        if not k or not c:
            raise SystemExit(f"{counter}: no samples for the kernel ({len(k)}) or the copy ({len(c)})")
        kk, cc = statistics.median(k), statistics.median(c)
        factor = a.copy_bytes / (cc * 1024.0)
        scaled = kk * 1024.0 * factor
        out[counter.lower()] = {"kernel_kib_per_dispatch": kk, "dispatches": len(k), "copy_kib": cc,
                                "copy_dispatches": len(c), "scale": factor, "bytes_per_launch": scaled}
        tot += scaled
    out["hbm_bytes_per_launch"] = tot
    out["algorithmic_bytes_per_launch"] = a.algorithmic_bytes
    out["traffic_over_algorithmic"] = tot / a.algorithmic_bytes
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def counter_table(path):
    """{(kernel, grid): {counter: [value per dispatch]}} of a counter-collection CSV."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            key = (short(_col(r, "Kernel_Name")), _grid(r))
            out.setdefault(key, {}).setdefault(_col(r, "Counter_Name"), []).append(float(_col(r, "Counter_Value")))
    return out


# per-wave ratios: (label, numerator, denominator)
SQ_RATIOS = [("VALU instructions per wave", "SQ_INSTS_VALU", "SQ_WAVES"),
             ("LDS instructions per wave", "SQ_INSTS_LDS", "SQ_WAVES"),
             ("wave lifetime per wave (SQ_WAVE_CYCLES units)", "SQ_WAVE_CYCLES", "SQ_WAVES"),
             ("VALU busy / lifetime", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES"),
             ("waiting on any instruction / lifetime", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
             ("waiting on LDS / lifetime", "SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES"),
             ("LDS bank-conflict cycles per LDS instruction", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS")]


def counters(a):
    tab = counter_table(a.csv)
    lines = [f"# Counters per dispatch: {os.path.basename(a.out)}", "",
             "Command (from the repository root on the GPU box):", "", "```", a.command, "```", ""]
    found = 0
    for kname in a.kernel:
        grids = [g for (n, g) in tab if n == kname]
        g = a.grid if a.grid is not None or not grids else max(grids)
        cs = tab.get((kname, g))
        if not cs:
            lines += [f"No dispatches of `{kname}`" + ("" if g is None else f" at grid {g}") + ".", ""]
            continue
        found += 1
        mean = {c: statistics.mean(v) for c, v in cs.items()}
        lines += [f"## `{kname}` at grid {g} ({max(len(v) for v in cs.values())} dispatches)", "",
                  "| counter | mean per dispatch |", "|---|---:|"]
        lines += [f"| {c} | {mean[c]:.6g} |" for c in sorted(mean)]
        rat = [(lab, mean[n] / mean[d]) for lab, n, d in SQ_RATIOS if n in mean and d in mean and mean[d] > 0]
        if rat:
            lines += ["", "| ratio | value |", "|---|---:|"] + [f"| {lab} | {v:.4g} |" for lab, v in rat]
        lines.append("")
    if not found:
        raise SystemExit("none of the kernels was dispatched")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--kernel", action="append", help="kernel name (repeatable; the first is the roofline kernel)")
    s.add_argument("--grid", type=int)
    s.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int)
    t.add_argument("--copy-kernel", default="elementwise|copy")
    t.add_argument("--copy-grid", type=int)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--sources", nargs="+", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--grid", type=int)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main(sys.argv[1:])
