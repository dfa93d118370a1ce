"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as Markdown.

  python -m paper_2604_26441_amd.profsummary RESULTS_DB [--match NAME --last N]

Prints the per-kernel totals (calls, total, average, share) and, with
--match, the average duration of the last N dispatches whose kernel name
contains NAME (for example the back-to-back timing loop of one kernel).
"""
import argparse
import sqlite3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--match", default=None)
    ap.add_argument("--last", type=int, default=200)
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
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
