"""Summaries of rocprofv3 CSV output (kernel statistics and hardware counters)
as Markdown tables, for the operator's kernels.

    python -m paper_1501_02946_amd.profiling stats <prefix>_kernel_stats.csv
    python -m paper_1501_02946_amd.profiling counters <prefix>_counter_collection.csv

Host-side text processing only: nothing here touches the GPU or the library.
"""
from __future__ import annotations

import csv
import re
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    """Kernel name without the return type, namespace and argument list; the
    template arguments are kept (they name the instantiation)."""
    n = name.strip().strip('"')
    n = re.sub(r"^void\s+", "", n)
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    return n.replace("nedner::", "").strip()


def base_name(name: str) -> str:
    """Kernel name without template arguments."""
    return short_name(name).split("<")[0]


def kernel_stats(path: str) -> list[dict]:
    """Rows of a rocprofv3 --stats kernel table: name, calls, average, minimum
    and maximum duration (µs) and share of the total kernel time (%)."""
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append(dict(name=short_name(r["Name"]), calls=int(r["Calls"]),
                             avg_us=float(r["AverageNs"]) / 1e3, min_us=float(r["MinNs"]) / 1e3,
                             max_us=float(r["MaxNs"]) / 1e3, share=float(r["Percentage"])))
    rows.sort(key=lambda r: -r["share"])
    return rows


def counter_means(path: str) -> dict:
    """Mean per dispatch of every counter of every kernel in a rocprofv3
    counter CSV: {kernel base name: {counter: (mean, dispatches)}}. Values of
    one counter within one dispatch (one row per hardware instance) are summed
    first."""
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            k = base_name(r["Kernel_Name"])
            per[k][r["Counter_Name"]][r.get("Dispatch_Id", r.get("Correlation_Id", ""))] += \
                float(r["Counter_Value"])
    out = {}
    for k, cs in per.items():
        out[k] = {c: (sum(d.values()) / len(d), len(d)) for c, d in cs.items()}
    return out


def stats_markdown(rows: list[dict], top: int = 24) -> str:
    lines = ["| kernel | calls | avg µs | min µs | max µs | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{r['name']}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | "
                     f"{r['max_us']:.1f} | {r['share']:.1f} |")
    return "\n".join(lines)


def counters_markdown(means: dict) -> str:
    names = sorted({c for cs in means.values() for c in cs})
    lines = ["| kernel | dispatches | " + " | ".join(names) + " |",
             "|---|---|" + "---|" * len(names)]
    for k in sorted(means):
        cs = means[k]
        n = max(v[1] for v in cs.values())
        lines.append(f"| `{k}` | {n} | " + " | ".join(f"{cs[c][0]:.4g}" if c in cs else "-"
                                                      for c in names) + " |")
    return "\n".join(lines)


def main(argv=None) -> int:
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 2 or argv[0] not in ("stats", "counters"):
        print(__doc__, file=sys.stderr)
        return 2
    if argv[0] == "stats":
        print(stats_markdown(kernel_stats(argv[1])))
    else:
        print(counters_markdown(counter_means(argv[1])))
    return 0


if __name__ == "__main__":
    sys.exit(main())
