"""Summarise rocprofv3 output into short markdown tables.

    python -m paper_2504_07090_amd.profsum stats <kernel_stats.csv> "<command>"
    python -m paper_2504_07090_amd.profsum counters <counter_collection.csv> "<command>"

`traffic_report` turns one FETCH_SIZE and one WRITE_SIZE run into HBM bytes
per launch, scaled by a device copy of known size at the end of each run.

`stats` lists the kernels by total GPU time; `counters` gives, per kernel,
the number of dispatches and the mean value of every collected counter per
dispatch (FETCH_SIZE and WRITE_SIZE are in KiB).
"""
import collections
import csv
import sys


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")[:70]


def summarise(path: str, command: str, top: int = 16, also=()) -> str:
    """The top kernels by total time, plus every kernel whose name contains one
    of the strings in ``also``."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    rows = rows[:top] + [r for r in rows[top:] if any(a in r["Name"] for a in also)]
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f} |")
    return "\n".join(out) + "\n"


def counter_means(path: str):
    """{kernel: {counter: mean per dispatch}} and {kernel: dispatches}."""
    vals = collections.defaultdict(lambda: collections.defaultdict(dict))
    for r in csv.DictReader(open(path)):
        k = _short(r["Kernel_Name"])
        d = vals[k][r["Counter_Name"]]
        did = r["Dispatch_Id"]
        d[did] = d.get(did, 0.0) + float(r["Counter_Value"])   # sum over dimensions of one dispatch
    means, calls = {}, {}
    for k, cs in vals.items():
        means[k] = {c: sum(v.values()) / len(v) for c, v in cs.items()}
        calls[k] = max(len(v) for v in cs.values())
    return means, calls


def summarise_counters(path: str, command: str, top: int = 20) -> str:
    means, calls = counter_means(path)
    names = sorted({c for m in means.values() for c in m})
    ks = sorted(means, key=lambda k: -max(means[k].values()))[:top]
    out = ["# rocprofv3 counters (mean per dispatch)", "", "Command:", "", "```", command, "```", "",
           "| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---:|" + "---:|" * len(names)]
    for k in ks:
        out.append(f"| `{k}` | {calls[k]} | " + " | ".join(f"{means[k].get(c, 0.0):.1f}" for c in names) + " |")
    return "\n".join(out) + "\n"


def traffic_report(fetch_csv: str, write_csv: str, command: str, kernels, sha: str,
                   copy_kib: float = 262144.0):
    """Markdown report of HBM bytes per launch from one FETCH_SIZE and one
    WRITE_SIZE run, each scaled by what the counter reads for the run's last
    dispatch, a device copy of copy_kib KiB read and written."""
    def last_copy(path):
        rows = [r for r in csv.DictReader(open(path)) if r["Kernel_Name"] == "__amd_rocclr_copyBuffer"]
        return float(rows[-1]["Counter_Value"])
    cf, cw = last_copy(fetch_csv), last_copy(write_csv)
    ff, fw = copy_kib / cf, copy_kib / cw
    fm, fn = counter_means(fetch_csv)
    wm, _ = counter_means(write_csv)
    out = ["# HBM traffic of the evaluation kernels (61-dish workload)", "",
           "Counters from two rocprofv3 runs, one per counter:", "", "```",
           command.format(C="FETCH_SIZE"), command.format(C="WRITE_SIZE"), "```", "",
           f"The last dispatch of each run is a {copy_kib / 1024:.0f} MiB device-to-device copy "
           "(`--calibrate-copy`), read and written once:", "",
           "| counter | copy reads as (KiB) | scale factor |", "|---|---:|---:|",
           f"| FETCH_SIZE | {cf:.1f} | {ff:.3f} |", f"| WRITE_SIZE | {cw:.1f} | {fw:.3f} |", "",
           "Per dispatch (means over the run; KiB as read, bytes after scaling):", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch (scaled) |",
           "|---|---:|---:|---:|---:|"]
    per = {}
    for k in kernels:
        if k not in fm:
            continue
        f, wv = fm[k]["FETCH_SIZE"], wm.get(k, {}).get("WRITE_SIZE", 0.0)
        b = (f * ff + wv * fw) * 1024
        per[k] = b
        out.append(f"| `{k}` | {fn[k]} | {f:.1f} | {wv:.1f} | {b:.4g} |")
    out += ["", f"Fringe kernel sources (fringe.hip, common.hpp) sha256 at the time of the runs: `{sha}`.", ""]
    return "\n".join(out) + "\n", per


def mfma_report(path: str, command: str, kernels, n_xcd: int = 8, n_simd: int = 1024) -> str:
    """Markdown table of MFMA and VALU activity per dispatch from one counter run
    (SQ_VALU_MFMA_BUSY_CYCLES, SQ_VALU_MFMA_COEXEC_CYCLES, SQ_INSTS_VALU,
    SQ_INSTS_MFMA, GRBM_GUI_ACTIVE).  The CSV sums GRBM_GUI_ACTIVE over the
    XCDs; divided by n_xcd it is the dispatch's active cycles, and
    MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x n_simd)."""
    m, n = counter_means(path)
    out = ["# MFMA and VALU activity of the fringe kernels (61-dish workload)", "",
           "Counters from one rocprofv3 run:", "", "```", command, "```", "",
           f"Active cycles = GRBM_GUI_ACTIVE / {n_xcd} (the CSV sums it over the XCDs); "
           f"MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x {n_simd} SIMDs).", "",
           "| kernel | dispatches | MFMA instr | VALU instr | VALU per MFMA | active cycles | "
           "MFMA busy | MFMA+VALU co-issue cycles |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in kernels:
        if k not in m:
            continue
        v = m[k]
        act = v["GRBM_GUI_ACTIVE"] / n_xcd
        busy = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (act * n_simd)
        mf = v["SQ_INSTS_MFMA"]
        out.append(f"| `{k}` | {n[k]} | {mf:.4g} | {v['SQ_INSTS_VALU']:.4g} | "
                   f"{v['SQ_INSTS_VALU'] / mf if mf else float('nan'):.2f} | {act:.4g} | {100 * busy:.1f}% | "
                   f"{v['SQ_VALU_MFMA_COEXEC_CYCLES']:.0f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    # stats <csv> <command> [top] [name substrings always listed ...]
    mode, path, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    if mode == "stats":
        top = int(sys.argv[4]) if len(sys.argv) > 4 else 16
        print(summarise(path, cmd, top, tuple(sys.argv[5:])))
    else:
        print(summarise_counters(path, cmd))
