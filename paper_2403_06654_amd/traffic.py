"""Turn two rocprofv3 --pmc runs of `bench.py --workload pmc` (256^3) or
`--workload pmc5` (512^3) (FETCH_SIZE, then WRITE_SIZE) into calibrated HBM
bytes per launch of the timed kernel classes, stored in
profiles/traffic_counters.json (256^3) or profiles/traffic_counters_c5.json
(512^3) for bench.py's roofline.

    python -m paper_2403_06654_amd.traffic FETCH_DIR WRITE_DIR [512]
    python -m paper_2403_06654_amd.traffic --md COUNTERS_JSON BENCH_JSON OUT.md TITLE COMMAND...

Calibration: the first device copy of the run moves exactly 1 GiB each way;
the ratio of that to what each counter reports for it scales every other
dispatch.  The result is keyed by a hash of the kernel sources so that it
is ignored once the kernels change.
"""
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

def class_patterns(n=256):
    """Kernel-name patterns of the timed classes on an n^3 grid (column
    passes of length n, row passes of n/2 complex points)."""
    c, r = n, n // 2
    return {
        "gmres gram-schmidt update (k_gs_update)": r"^void vd::k_gs_update<double,",
        "gmres gram-schmidt dots (k_mdot)": r"^void vd::k_mdot<double, (?!1>)",
        "pressure x pass (k_row ROW_P)": rf"^void vd::k_row<{r}, double, 2>",
        "pressure z-first (k_col COL_P_FIRST)": rf"^void vd::k_col<{c}, double, 2>",
        "pressure y-inverse (k_col COL_P_MIDINV)": rf"^void vd::k_col<{c}, double, 3>",
        "pressure y-forward (k_col COL_P_MIDFWD)": rf"^void vd::k_col<{c}, double, 4>",
        "pressure z-last (k_col COL_P_LAST)": rf"^void vd::k_col<{c}, double, 5>",
        "helmholtz z-first (k_col COL_H_FIRST)": rf"^void vd::k_col<{c}, double, 6>",
        "y inverse FFT, one field (k_col COL_FFT_INV)": rf"^void vd::k_col<{c}, double, 1>",
        "helmholtz x pass (k_row ROW_H)": rf"^void vd::k_row<{r}, double, 4>",
        "y forward FFT, one field (k_col COL_FFT_FWD)": rf"^void vd::k_col<{c}, double, 0>",
        "helmholtz z-last (k_col COL_H_LAST)": rf"^void vd::k_col<{c}, double, 7>",
        # FP32 operator passes (the inner solves of iterative refinement)
        "fp32 pressure z-first (k_col COL_P_FIRST)": rf"^void vd::k_col<{c}, float, 2>",
        "fp32 pressure y-inverse (k_col COL_P_MIDINV)": rf"^void vd::k_col<{c}, float, 3>",
        "fp32 pressure x pass (k_row ROW_P)": rf"^void vd::k_row<{r}, float, 2>",
        "fp32 pressure y-forward (k_col COL_P_MIDFWD)": rf"^void vd::k_col<{c}, float, 4>",
        "fp32 pressure z-last (k_col COL_P_LAST)": rf"^void vd::k_col<{c}, float, 5>",
    }


CLASS_PATTERNS = class_patterns(256)


def _rows(d):
    path = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    return list(csv.DictReader(open(path)))


def summarize(F, W, source_hash, patterns=None):
    """Calibrated per-launch HBM bytes of the timed kernel classes from the
    FETCH_SIZE rows F and the WRITE_SIZE rows W (rocprofv3 counter CSV rows,
    in dispatch order)."""
    copy_bytes = 1 << 30
    cf = next(r for r in F if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"))
    cw = next(r for r in W if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"))
    kf = copy_bytes / (float(cf["Counter_Value"]) * 1024)
    kw = copy_bytes / (float(cw["Counter_Value"]) * 1024)
    out = {"csrc_sha256_16": source_hash, "calibration": {"copy_bytes": copy_bytes, "fetch_factor": kf,
                                                           "write_factor": kw},
           "per_launch_bytes": {}, "launches": {}}
    for name, pat in (patterns or CLASS_PATTERNS).items():
        fv = [float(r["Counter_Value"]) * 1024 * kf for r in F if re.match(pat, r["Kernel_Name"])]
        wv = [float(r["Counter_Value"]) * 1024 * kw for r in W if re.match(pat, r["Kernel_Name"])]
        if fv and len(fv) == len(wv):
            # A Krylov step queued past the end of its run launches every
            # kernel, which returns at its gate having read a flag only: such
            # dispatches (under 1% of the median traffic) are not launches of
            # the timed work and are left out, as the HIP-event timing does.
            med = sorted(fv)[len(fv) // 2]
            keep = [i for i in range(len(fv)) if fv[i] >= 0.01 * med]
            out["per_launch_bytes"][name] = round(sum(fv[i] + wv[i] for i in keep) / len(keep))
            out["launches"][name] = len(keep)
            out.setdefault("gated_dispatches_left_out", {})[name] = len(fv) - len(keep)
    return out


def main(fetch_dir, write_dir, n=256):
    from bench import csrc_hash  # noqa: E402
    out = summarize(_rows(fetch_dir), _rows(write_dir), csrc_hash(), class_patterns(n))
    out["grid"] = n
    name = "traffic_counters.json" if n == 256 else f"traffic_counters_c{5 if n == 512 else n}.json"
    path = os.path.join(ROOT, "profiles", name)
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


# fields each pass moves (F = one half-spectrum field of the grid's precision)
PASS_FIELDS = {"pressure z-first (k_col COL_P_FIRST)": 3, "pressure y-inverse (k_col COL_P_MIDINV)": 5,
               "pressure x pass (k_row ROW_P)": 7, "pressure y-forward (k_col COL_P_MIDFWD)": 5,
               "pressure z-last (k_col COL_P_LAST)": 3, "helmholtz z-first (k_col COL_H_FIRST)": 2,
               "y inverse FFT, one field (k_col COL_FFT_INV)": 2, "helmholtz x pass (k_row ROW_H)": 3,
               "y forward FFT, one field (k_col COL_FFT_FWD)": 2, "helmholtz z-last (k_col COL_H_LAST)": 3}


def markdown(t, bench_line, commands, title):
    """profiles/ summary of a counter summary t (the JSON main writes) beside
    the algorithmic bytes per launch: the roofline kernel's from the bench
    line, every pass's from its field count."""
    n = t["grid"]
    F = n * n * (n // 2) * 16
    alg = {}
    rf = (bench_line or {}).get("roofline") or {}
    if rf.get("kernel"):
        alg[rf["kernel"]] = rf["bytes_per_launch"]
    lines = [f"# {title}", "", "Commands (repository root, one MI355X), one counter per pass:", "", "```"]
    lines += commands + ["```", "",
                         f"Calibration (1 GiB device copy): fetched bytes scaled by "
                         f"{t['calibration']['fetch_factor']:.4f}, written bytes by {t['calibration']['write_factor']:.3f}. "
                         f"F = one FP64 half-spectrum field = {F:,} B (FP32: F/2).", "",
                         "| kernel class | fields moved | algorithmic bytes / launch | calibrated FETCH+WRITE / launch | "
                         "ratio | launches | gated, left out |", "|---|---:|---:|---:|---:|---:|---:|"]
    for name, v in t["per_launch_bytes"].items():
        base = name[5:] if name.startswith("fp32 ") else name
        a, fl = alg.get(name), "(nv+2)F per system" if "update" in name else "(nv+1)F per system"
        if base in PASS_FIELDS:
            k = PASS_FIELDS[base]
            a = k * F // (2 if name.startswith("fp32 ") else 1)
            fl = f"{k}F" + ("/2" if name.startswith("fp32 ") else "")
        ratio = f"{v / a:.4f}" if a else "n/a"
        lines.append(f"| {name} | {fl} | {f'{a:,}' if a else 'n/a'} | {v:,} | {ratio} | {t['launches'][name]} | "
                     f"{t.get('gated_dispatches_left_out', {}).get(name, 0)} |")
    lines += ["", f"Kernel-source hash `{t['csrc_sha256_16']}`: bench.py reports `roofline.traffic` from the JSON beside "
              "this file only while the sources match.", ""]
    return "\n".join(lines)


if __name__ == "__main__":
    if "--md" in sys.argv:
        # python -m paper_2403_06654_amd.traffic --md COUNTERS_JSON BENCH_JSON OUT.md TITLE COMMAND...
        i = sys.argv.index("--md")
        cj, bj, out, title = sys.argv[i + 1:i + 5]
        bench = json.loads(open(bj).read().strip().splitlines()[-1]) if bj != "-" else None
        open(out, "w").write(markdown(json.load(open(cj)), bench, sys.argv[i + 5:], title))
        print(out)
    else:
        main(sys.argv[1], sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 256)
