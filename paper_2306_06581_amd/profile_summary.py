"""Summaries of rocprofv3 CSV output (``--output-format csv``).

    python -m paper_2306_06581_amd.profile_summary stats DIR [--top N] [--kernel SUBSTR]
        per-kernel dispatch count, total / mean / min / max duration, from the
        kernel trace (End - Start of every dispatch)
    python -m paper_2306_06581_amd.profile_summary pmc DIR --kernel SUBSTR
        per-dispatch mean / min / max of every collected counter for the
        kernels whose name contains SUBSTR

DIR is the ``-d`` directory of a rocprofv3 run; files are found recursively.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import statistics
from collections import defaultdict


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def kernel_durations(d: str) -> dict[str, list[float]]:
    """Kernel name -> durations of its dispatches in microseconds."""
    out: dict[str, list[float]] = defaultdict(list)
    for r in _rows(d, "kernel_trace.csv"):
        out[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return out


def stats(d: str, top: int = 20, kernel: str | None = None) -> str:
    dur = kernel_durations(d)
    if kernel:
        dur = {k: v for k, v in dur.items() if kernel in k}
    total = sum(sum(v) for v in dur.values()) or 1.0
    lines = ["| kernel | calls | total us | mean us | min us | max us | share |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:top]:
        short = name if len(name) <= 90 else name[:87] + "..."
        lines.append(f"| `{short}` | {len(v)} | {sum(v):.1f} | {statistics.fmean(v):.2f} | "
                     f"{min(v):.2f} | {max(v):.2f} | {100 * sum(v) / total:.1f}% |")
    return "\n".join(lines)


def pmc(d: str, kernel: str) -> str:
    vals: dict[str, list[float]] = defaultdict(list)
    for r in _rows(d, "counter_collection.csv"):
        if kernel in r["Kernel_Name"]:
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {kernel!r}")
    lines = ["| counter | dispatches | mean | min | max |", "|---|---:|---:|---:|---:|"]
    for c, v in sorted(vals.items()):
        lines.append(f"| {c} | {len(v)} | {statistics.fmean(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc"])
    ap.add_argument("dir")
    ap.add_argument("--kernel")
    ap.add_argument("--top", type=int, default=20)
    a = ap.parse_args()
    if a.mode == "stats":
        print(stats(a.dir, a.top, a.kernel))
    else:
        if not a.kernel:
            raise SystemExit("pmc needs --kernel")
        print(pmc(a.dir, a.kernel))


if __name__ == "__main__":
    main()
