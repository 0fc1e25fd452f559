"""Markdown summary of a rocprofv3 `--kernel-trace --stats` run, for
profiles/: the kernels that took the most time, and for every timed kernel
class of an n^3 grid the average duration of its dispatches that did work,
set beside the HIP-event figures of a bench.py JSON line.

A Krylov step that the solver queued past the end of its run launches its
kernels, which read one device flag and return; bench.py's HIP-event timing
drops those launches, and so does this summary (dispatches shorter than
GATE_US, far below any working launch at these sizes).

    python -m paper_2403_06654_amd.profsum PROF_DIR BENCH_JSON N OUT.md TITLE COMMAND [TOP]

BENCH_JSON "-": no class table (a run on other grids than n^3).
"""
import csv
import glob
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2403_06654_amd.traffic import class_patterns  # noqa: E402

GATE_US = 10.0


def _csv(d, suffix):
    path = glob.glob(os.path.join(d, f"*{suffix}"))[0]
    return list(csv.DictReader(open(path)))


def class_durations(trace, patterns):
    """Per class: durations (us) of the dispatches that did work, and the
    number of gated ones."""
    out = {}
    for name, pat in patterns.items():
        rx = re.compile(pat)
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace if rx.match(r["Kernel_Name"])]
        work = [x for x in d if x >= GATE_US]
        out[name] = (work, len(d) - len(work))
    return out


# bench.py's names of the classes that the counter patterns name otherwise
ALIASES = {"helmholtz y-inverse (k_col COL_FFT_INV)": "y inverse FFT, one field (k_col COL_FFT_INV)",
           "helmholtz y-forward (k_col COL_FFT_FWD)": "y forward FFT, one field (k_col COL_FFT_FWD)"}


def bench_figures(line):
    """Class name -> (avg us, launches) from a bench.py JSON line: its
    per-pass table and its roofline kernel."""
    fig = {}
    for name, p in (line.get("passes") or {}).items():
        fig[ALIASES.get(name, name)] = (p["avg_us"], p["launches"], "warm-up steps")
    rf = line.get("roofline") or {}
    if rf.get("kernel"):
        fig[rf["kernel"]] = (rf["avg_launch_us"], rf["launches"], "timed steps (roofline)")
    return fig


def render(prof_dir, bench_line, n, title, command, top=20):
    stats = _csv(prof_dir, "kernel_stats.csv")
    # the per-dispatch trace (large) may be left out of a run: then totals only
    trace = _csv(prof_dir, "kernel_trace.csv") if glob.glob(os.path.join(prof_dir, "*kernel_trace.csv")) else []
    total_ms = sum(float(r["TotalDurationNs"]) for r in stats) / 1e6
    lines = [f"# {title}", "", "Command (repository root, one MI355X):", "", "```", command, "```", "",
             f"Per-kernel totals from rocprofv3 `--stats`, top {top} by time:", "",
             "| % time | calls | avg us | kernel |", "|---:|---:|---:|---|"]
    for r in stats[:top]:
        lines.append(f"| {float(r['Percentage']):.2f} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"`{r['Name'][:110]}` |")
    lines += ["", f"Total kernel time: {total_ms:.1f} ms.", ""]
    if bench_line is None:  # no bench line: kernels of other shapes than the n^3 classes
        return "\n".join(lines + gemm_shapes(trace)) + "\n"
    durs = class_durations(trace, class_patterns(n))
    fig = bench_figures(bench_line)
    lines += [f"Timed kernel classes: average over the dispatches that did work (gated dispatches, shorter "
              f"than {GATE_US:g} us, left out and counted apart), beside bench.py's HIP-event figure for the class:", "",
              "| kernel class | rocprofv3 avg us (launches) | median us | gated | bench.py avg us (launches, where) | "
              "difference |", "|---|---:|---:|---:|---:|---:|"]
    for name, (work, gated) in durs.items():
        if not work:
            continue
        avg = sum(work) / len(work)
        b = fig.get(name)
        bs = f"{b[0]:.2f} ({b[1]}, {b[2]})" if b else "n/a"
        diff = f"{100.0 * (avg - b[0]) / b[0]:+.1f}%" if b else ""
        lines.append(f"| {name} | {avg:.2f} ({len(work)}) | {statistics.median(work):.2f} | {gated} | {bs} | {diff} |")
    lines.append("")
    lines += gemm_shapes(trace)
    return "\n".join(lines) + "\n"


def gemm_shapes(trace):
    """The Chebyshev contractions (k_gemm) by launch shape: one 16 x 16 tile
    of C per block, so the grid gives M (rows, 16 per block row) and N."""
    groups = {}
    for r in trace:
        name = r["Kernel_Name"]
        if "k_gemm" not in name:
            continue
        key = (name.split("(")[0], int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]), int(r["Grid_Size_Y"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    if not groups:
        return []
    out = ["Chebyshev contractions (k_gemm) by launch shape: durations of the dispatches that did work "
           "(gated ones, shorter than 3 us, left out), percentiles in us:", "",
           "| kernel | column tiles x row tiles | launches | p10 | p25 | p50 | p75 | p90 |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (name, nx, ny), d in sorted(groups.items()):
        w = sorted(x for x in d if x >= 3.0)
        if not w:
            continue
        q = [w[min(len(w) - 1, int(f * len(w)))] for f in (0.10, 0.25, 0.50, 0.75, 0.90)]
        out.append(f"| `{name}` | {nx} x {ny} | {len(w)} | " + " | ".join(f"{x:.2f}" for x in q) + " |")
    out.append("")
    return out


def main(argv):
    prof_dir, bench_json, n, out, title, command = argv[:6]
    top = int(argv[6]) if len(argv) > 6 else 20
    line = None
    if bench_json != "-":
        text = open(bench_json).read().strip().splitlines()
        line = json.loads(text[-1])
    md = render(prof_dir, line, int(n), title, command, top)
    open(out, "w").write(md)
    print(out)


if __name__ == "__main__":
    main(sys.argv[1:])
