"""Summarise rocprofv3 output into short markdown tables.

    python -m paper_2504_07090_amd.profsum stats <kernel_stats.csv> "<command>"
    python -m paper_2504_07090_amd.profsum counters <counter_collection.csv> "<command>"

`stats` lists the kernels by total GPU time; `counters` gives, per kernel,
the number of dispatches and the mean value of every collected counter per
dispatch (FETCH_SIZE and WRITE_SIZE are in KiB).
"""
import collections
import csv
import sys


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")[:70]


def summarise(path: str, command: str, top: int = 16) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
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


if __name__ == "__main__":
    mode, path, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    print(summarise(path, cmd) if mode == "stats" else summarise_counters(path, cmd))
