"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as Markdown.

  python -m paper_2604_26441_amd.profsummary RESULTS_DB [--match NAME --last N]
  python -m paper_2604_26441_amd.profsummary --counters COUNTER_CSV

Prints the per-kernel totals (calls, total, average, share) and, with
--match, the average duration of the last N dispatches whose kernel name
contains NAME (for example the back-to-back timing loop of one kernel).
With --counters, reads a rocprofv3 --pmc CSV (counter_collection.csv) and
prints, per kernel, the dispatch count and the mean of each counter.
"""
import argparse
import csv
import sqlite3
from collections import defaultdict


def counters(path):
    acc = defaultdict(lambda: defaultdict(list))
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name", "").replace("sgmg::", "").split("(")[0]
            acc[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
    cols = sorted({c for k in acc.values() for c in k})
    print("| kernel | dispatches | " + " | ".join(f"mean {c}" for c in cols) + " |")
    print("|---|---|" + "---|" * len(cols))
    for name, byc in acc.items():
        nd = max(len(v) for v in byc.values())
        vals = [sum(byc[c]) / len(byc[c]) if byc[c] else float("nan") for c in cols]
        print(f"| `{name}` | {nd} | " + " | ".join(f"{v:.1f}" for v in vals) + " |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--counters", default=None)
    ap.add_argument("--match", default=None)
    ap.add_argument("--last", type=int, default=200)
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
    if a.counters:
        counters(a.counters)
        return
    c = sqlite3.connect(a.db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels"))
    print("| kernel | calls | total (ms) | average (us) | share |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows[: a.top]:
        short = name.replace("sgmg::", "").split("(")[0]
        print(f"| `{short}` | {calls} | {tot / 1e3:.3f} | {avg:.3f} | {pct:.1f}% |")
    if a.match:
        durs = [r[0] for r in c.execute(
            "select duration from kernels where name like ? order by start", (f"%{a.match}%",))]
        last = durs[-a.last:]
        if last:
            print(f"\nLast {len(last)} dispatches matching `{a.match}`: average "
                  f"{sum(last) / len(last) / 1e3:.3f} us, min {min(last) / 1e3:.3f} us, "
                  f"max {max(last) / 1e3:.3f} us")


if __name__ == "__main__":
    main()
