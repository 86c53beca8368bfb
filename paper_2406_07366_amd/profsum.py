"""Text summaries of rocprofv3 output for the measurement record.

  python -m paper_2406_07366_amd.profsum stats <kernel_stats.csv> <out.txt> <command...>
      per-kernel call counts and mean durations (from --kernel-trace --stats)

  python -m paper_2406_07366_amd.profsum pmc <kernel-regex> <fetch.csv> <write.csv>
          <copy_bytes> <source.hip> <out.txt> <command...>
      HBM bytes per launch of the kernels matching <kernel-regex>, from two
      --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the
      ratio of the known size of the largest plain device copy in the same
      run to what the same counter reads for it.  The summary records the
      SHA-1 of the kernel's source file: a reader compares it with the file as
      it stands and ignores the figure once the source has changed.

The bench reads `traffic_bytes_per_launch` and `source_sha1` back from the
pmc summary (see read_traffic).
"""
from __future__ import annotations

import csv
import hashlib
import re
import sys


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats(csv_path, out_path, command):
    rows = _rows(csv_path)
    lines = [f"# rocprofv3 kernel statistics", f"command: {command}", "",
             f"{'kernel':<96s} {'calls':>6s} {'mean_us':>10s} {'total_%':>8s}"]
    for r in rows:
        name = r["Name"]
        name = name if len(name) <= 96 else name[:93] + "..."
        lines.append(f"{name:<96s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):8.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    """(kernel name, value) per dispatch for one counter."""
    out = {}
    for r in _rows(path):
        if r.get("Counter_Name", "") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        out[key] = (r["Kernel_Name"], float(r["Counter_Value"]))
    return list(out.values())


def sha1_of(path):
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def pmc(regex, fetch_csv, write_csv, copy_bytes, source, out_path, command):
    pat = re.compile(regex)
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = _per_dispatch(path, counter)
        copies = [v for n, v in d if "copyBuffer" in n]
        kern = [v for n, v in d if pat.search(n)]
        if not copies or not kern:
            raise SystemExit(f"{counter}: no copy ({len(copies)}) or kernel ({len(kern)}) dispatches")
        cal = max(copies)                       # KiB for copy_bytes moved
        factor = (copy_bytes / 1024.0) / cal
        mean = sum(kern) / len(kern)
        res[counter] = dict(raw_kib=mean, copy_kib=cal, factor=factor,
                            bytes=mean * 1024.0 * factor, n=len(kern))
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    lines = ["# rocprofv3 PMC traffic (HBM bytes per launch)",
             f"command (one run per counter): {command}",
             f"kernel regex: {regex}", f"calibration: largest device copy of {copy_bytes} B", ""]
    for c, r in res.items():
        lines.append(f"{c}: {r['raw_kib']:.1f} KiB per dispatch over {r['n']} dispatches; "
                     f"copy reads {r['copy_kib']:.1f} KiB, factor {r['factor']:.4f}, "
                     f"{r['bytes']:.4e} B")
    lines += [f"traffic_bytes_per_launch: {total:.6e}", f"source: {source}",
              f"source_sha1: {sha1_of(source)}"]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_traffic(summary_path, source_path):
    """HBM bytes per launch from a pmc summary, or None if it is missing or
    its kernel source has changed since the counters were taken."""
    try:
        txt = open(summary_path).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\S+)", txt)
    h = re.search(r"source_sha1: (\S+)", txt)
    if not m or not h or h.group(1) != sha1_of(source_path):
        return None
    return float(m.group(1))


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "stats":
        stats(a[1], a[2], " ".join(a[3:]))
    elif a and a[0] == "pmc":
        pmc(a[1], a[2], a[3], float(a[4]), a[5], a[6], " ".join(a[7:]))
    else:
        raise SystemExit(__doc__)
