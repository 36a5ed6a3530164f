"""Summaries of rocprofv3 CSV output for the text files under profiles/.

    python -m paper_1507_01391_amd.profile_summary kernels <kernel_stats.csv>
    python -m paper_1507_01391_amd.profile_summary counters <counter_collection.csv> [...] --steps S

``kernels`` prints the per-kernel time table of a ``--kernel-trace --stats`` run;
``counters`` sums every counter of one or more ``--pmc`` runs per kernel, over all its
dispatches and per step (the workload ran ``--steps`` times: profile_run's untimed
launch plus its repetitions).
"""
from __future__ import annotations

import argparse
import csv
import re
from collections import defaultdict


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"^void ", "", name)
    depth, out = 0, []
    for ch in name:           # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def kernels(path: str) -> None:
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"| kernel | calls | total ms | average us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        print(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
              f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.1f} |")


def counters(paths, steps: int) -> None:
    sums = defaultdict(float)
    disp = defaultdict(set)
    names = []
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            c = r["Counter_Name"]
            sums[(k, c)] += float(r["Counter_Value"])
            disp[k].add((path, r.get("Dispatch_Id") or r.get("Correlation_Id")))
            if c not in names:
                names.append(c)
    kern = sorted(disp, key=lambda k: -sum(sums[(k, c)] for c in names))
    print("| kernel | dispatches | " + " | ".join(f"{c} per step" for c in names) + " |")
    print("|---|---|" + "---|" * len(names))
    total = defaultdict(float)
    for k in kern:
        vals = []
        for c in names:
            v = sums[(k, c)] / steps
            total[c] += v
            vals.append(f"{v:,.0f}")
        print(f"| `{k}` | {len(disp[k])} | " + " | ".join(vals) + " |")
    print("| **all kernels** | | " + " | ".join(f"**{total[c]:,.0f}**" for c in names) + " |")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("kernels")
    p.add_argument("csv")
    p = sub.add_parser("counters")
    p.add_argument("csv", nargs="+")
    p.add_argument("--steps", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        kernels(a.csv)
    else:
        counters(a.csv, a.steps)


if __name__ == "__main__":
    main()
