"""Summarise rocprofv3 CSV output of a bench.py run (kernel trace and counters).

    python -m paper_2202_02264_amd.rocprof_summary --trace T_kernel_trace.csv \
        --stats T_kernel_stats.csv --match 'k_rows' --last 60 \
        [--fetch F.csv --write W.csv --last-counted 24 --copy-fetch CF.csv --copy-write CW.csv]

--last keeps the last N dispatches whose name matches --match (the timed steps
of the run; earlier ones include warm-up and tile autotuning) and prints their
average duration.  FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the last
--last-counted matching dispatches are scaled by what the same counters read
for a device copy of known size (copy-calibration run of bench.py: 10 copies
of 256 MiB, each reading and writing 256 MiB).
"""
from __future__ import annotations

import argparse
import csv
import re
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def stats_table(path: str, top: int = 12) -> str:
    rows = _rows(path)
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def timed_average(trace: str, match: str, last: int):
    rx = re.compile(match)
    d = [r for r in _rows(trace) if rx.search(r["Kernel_Name"])]
    d.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = d[-last:] if last else d
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in d]
    by = defaultdict(list)
    for r, t in zip(d, durs):
        by[_short(r["Kernel_Name"])].append(t)
    return len(durs), sum(durs) / max(1, len(durs)), {k: (len(v), sum(v) / len(v)) for k, v in by.items()}


def counter_per_dispatch(path: str, match: str, last: int, counter: str):
    rx = re.compile(match)
    d = [r for r in _rows(path) if rx.search(r["Kernel_Name"]) and r["Counter_Name"] == counter]
    d.sort(key=lambda r: int(r["Dispatch_Id"]))
    d = d[-last:] if last else d
    vals = [float(r["Counter_Value"]) for r in d]
    return len(vals), sum(vals) / max(1, len(vals))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--stats")
    ap.add_argument("--match", required=True)
    ap.add_argument("--last", type=int, default=0)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--last-counted", type=int, default=0)
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    a = ap.parse_args()
    if a.stats:
        print("rocprofv3 --stats (all dispatches of the run, warm-up and autotuning included):\n")
        print(stats_table(a.stats))
        print()
    n, avg, by = timed_average(a.trace, a.match, a.last)
    print(f"timed region: last {n} dispatches matching `{a.match}`: average {avg / 1e3:.2f} us")
    for k, (c, v) in sorted(by.items()):
        print(f"  {k}: {c} dispatches, average {v / 1e3:.2f} us")
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        copy_kib = 256 * 1024.0
        _, cf = counter_per_dispatch(a.copy_fetch, "copyBuffer", 0, "FETCH_SIZE")
        _, cw = counter_per_dispatch(a.copy_write, "copyBuffer", 0, "WRITE_SIZE")
        sf, sw = copy_kib / cf, copy_kib / cw
        nf, f = counter_per_dispatch(a.fetch, a.match, a.last_counted, "FETCH_SIZE")
        nw, w = counter_per_dispatch(a.write, a.match, a.last_counted, "WRITE_SIZE")
        print(f"\ncopy calibration (256 MiB read + 256 MiB written per dispatch): FETCH_SIZE reads "
              f"{cf:.0f} KiB (scale {sf:.3f}), WRITE_SIZE reads {cw:.0f} KiB (scale {sw:.3f})")
        print(f"last {nf} dispatches matching `{a.match}`: FETCH_SIZE {f:.0f} KiB -> {f * sf / 1024:.2f} MiB "
              f"read, WRITE_SIZE {w:.0f} KiB -> {w * sw / 1024:.2f} MiB written per dispatch "
              f"(HBM traffic {(f * sf + w * sw) * 1024 / 1e6:.2f} MB per dispatch)")


if __name__ == "__main__":
    main()
