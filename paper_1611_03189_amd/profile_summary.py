"""Condense a rocprofv3 ``--stats`` kernel table (``*_kernel_stats.csv``) into the short text
summary kept beside the measurements: one line per kernel with calls, total and mean time.

    python -m paper_1611_03189_amd.profile_summary STATS_CSV "COMMAND" [TITLE] > summary.txt
"""
import csv
import sys


def summarize(path: str, command: str, title: str = "") -> str:
    rows = list(csv.DictReader(open(path)))
    out = []
    if title:
        out.append(f"# {title}")
    out.append(f"# command: {command}")
    out.append(f"# {'kernel':58s} {'calls':>6s} {'total_ms':>10s} {'mean_us':>10s} {'pct':>6s}")
    for r in rows:
        name = r["Name"]
        if "(" in name:
            name = name[:name.index("(")]
        name = name.replace("void ", "")
        out.append(f"  {name[:58]:58s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                   f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    print(summarize(sys.argv[1], sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""), end="")
