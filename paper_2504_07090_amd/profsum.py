"""Summarise a rocprofv3 kernel_stats.csv into a short markdown table.

    python -m paper_2504_07090_amd.profsum <kernel_stats.csv> "<command that produced it>"
"""
import csv
import sys


def summarise(path: str, command: str, top: int = 16) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name[:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    print(summarise(sys.argv[1], sys.argv[2]))
