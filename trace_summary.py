"""Summarise a rocprofv3 ``--kernel-trace --stats`` run as a markdown table.

Reads the run's ``*_kernel_stats.csv`` and writes a short markdown file with
the command, a description and one row per kernel (calls, total, average,
min and max in ns, share of the GPU time, and for full-sweep kernels the
GB/s at the average duration given the state size).

usage: python trace_summary.py STATS_CSV OUT_MD "TITLE" "COMMAND" "DESCRIPTION" [STATE_BYTES [SWEEP_KERNEL_SUBSTR ...]]
"""
from __future__ import annotations

import csv
import sys


def main(argv):
    if len(argv) < 6:
        print(__doc__)
        return 2
    stats, out, title, command, desc = argv[1:6]
    state_bytes = float(argv[6]) if len(argv) > 6 else 0.0
    sweep_names = argv[7:]
    rows = []
    with open(stats) as f:
        for r in csv.DictReader(f):
            rows.append(r)

    def col(r, *names):
        for n in names:
            if n in r:
                return r[n]
        raise KeyError(names)
    lines = ["# %s" % title, "", "Command: `%s`" % command, "", desc, "",
             "| kernel | calls | total | average | min | max | % | GB/s at average |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(col(r, "TotalDurationNs", "TotalDuration"))):
        name = col(r, "Name", "KernelName")
        short = name.replace("sv::(anonymous namespace)::", "").replace("sv::", "")
        if short.startswith("void "):
            short = short[5:]
        short = short.split("(")[0]
        avg = float(col(r, "AverageNs", "Average"))
        gbps = ""
        if state_bytes and any(s in short for s in sweep_names):
            gbps = "%.0f" % (2 * state_bytes / avg)
        lines.append("| `%s` | %s | %s | %.0f | %s | %s | %.2f | %s |" % (
            short, col(r, "Calls"), col(r, "TotalDurationNs", "TotalDuration"), avg, col(r, "MinNs", "Min"),
            col(r, "MaxNs", "Max"), float(col(r, "Percentage")), gbps))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
