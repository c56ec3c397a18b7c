"""Summarise rocprofv3 byte counters for the dominant sweep kernel.

Reads two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` CSV outputs
(``*_counter_collection.csv``) of ``bench.py --copy-probe`` runs, scales each
counter by what it reads for the plain device copy of the state's size
(the largest ``copyBuffer`` dispatch: known to move S bytes in and S out),
and writes the per-launch HBM bytes of the chosen kernel as JSON and
markdown.  The JSON carries the hash of the kernel source it was taken on;
bench.py reports the figure only while that source is unchanged.

usage: python pmc_summary.py FETCH_CSV WRITE_CSV KERNEL_SUBSTR STATE_BYTES OUT_STEM "COMMAND..." [SOURCE [ALG_BYTES]]

SOURCE is the kernel's source file under paper_2608_16940_amd/csrc (default sv_tile.hip).
ALG_BYTES is the algorithmic bytes per launch averaged over the counted
launches (default 2 * STATE_BYTES, a full sweep; less when some launches
touch part of the state, as controlled diagonal sweeps do).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2608_16940_amd", "csrc")


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def per_launch(path, kernel_substr):
    rows = _rows(path)
    vals = [float(r["Counter_Value"]) * 1024.0 for r in rows if kernel_substr in r["Kernel_Name"]]
    copies = [float(r["Counter_Value"]) * 1024.0 for r in rows if "copyBuffer" in r["Kernel_Name"]]
    return vals, max(copies) if copies else None


def main(argv):
    fetch_csv, write_csv, ksub, state_bytes, stem, cmd = argv[1:7]
    src = argv[7] if len(argv) > 7 else "sv_tile.hip"
    state_bytes = float(state_bytes)
    alg = float(argv[8]) if len(argv) > 8 else 2 * state_bytes
    fv, fcopy = per_launch(fetch_csv, ksub)
    wv, wcopy = per_launch(write_csv, ksub)
    fscale = state_bytes / fcopy
    wscale = state_bytes / wcopy
    f = statistics.mean(fv) * fscale
    w = statistics.mean(wv) * wscale
    with open(os.path.join(CSRC, src), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    out = {
        "kernel": ksub, "launches": len(fv), "source": src, "source_sha": sha,
        "fetch_bytes_per_launch": f, "write_bytes_per_launch": w, "bytes_per_launch": f + w,
        "fetch_scale_from_copy": fscale, "write_scale_from_copy": wscale,
        "copy_probe_bytes_each_way": state_bytes, "algorithmic_bytes_per_launch": alg, "command": cmd,
    }
    with open(stem + ".json", "w") as fh:
        json.dump(out, fh, indent=1)
    with open(stem + ".md", "w") as fh:
        fh.write("# HBM bytes per launch: %s\n\n" % ksub)
        fh.write("Command (run twice, with `--pmc FETCH_SIZE` and with `--pmc WRITE_SIZE`):\n\n```\n%s\n```\n\n" % cmd)
        fh.write("| quantity | value |\n|---|---|\n")
        fh.write("| launches counted | %d |\n" % len(fv))
        fh.write("| FETCH_SIZE raw mean | %.0f KiB |\n" % (statistics.mean(fv) / 1024))
        fh.write("| WRITE_SIZE raw mean | %.0f KiB |\n" % (statistics.mean(wv) / 1024))
        fh.write("| copy probe (%.0f B each way): FETCH_SIZE / WRITE_SIZE | %.0f / %.0f KiB |\n"
                 % (state_bytes, fcopy / 1024, wcopy / 1024))
        fh.write("| scale factors fetch / write | %.4f / %.4f |\n" % (fscale, wscale))
        fh.write("| HBM read bytes per launch | %.4e |\n" % f)
        fh.write("| HBM write bytes per launch | %.4e |\n" % w)
        fh.write("| total per launch | %.4e (algorithmic %.4e) |\n" % (f + w, alg))
        fh.write("| kernel source %s sha256[:16] | %s |\n" % (src, sha))
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv)
