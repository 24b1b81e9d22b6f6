"""Summarise a rocprofv3 kernel trace (rocpd SQLite output) per kernel.

    python -m paper_1307_4839_amd.rocprof_summary RESULTS.db [--skip NAME=K ...]

Prints, per kernel name: dispatch count, total and average duration over all
dispatches, and the average over the dispatches left after skipping the
first K dispatches of that kernel (``--skip``), e.g. the warmup steps of a
benchmark whose timed region starts after them.
"""

from __future__ import annotations

import argparse
import sqlite3
import sys


def summarize(db: str, skip: dict) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, duration from kernels order by start").fetchall()
    per = {}
    for name, start, dur in rows:
        per.setdefault(name, []).append(dur)
    out = []
    out.append(f"{'kernel':<60} {'calls':>6} {'total_ms':>10} {'avg_us':>10} "
               f"{'skip':>5} {'avg_us_after_skip':>18}")
    for name, durs in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        k = 0
        for key, val in skip.items():
            if key in name:
                k = val
        rest = durs[k:] if k < len(durs) else []
        avg_rest = (sum(rest) / len(rest) / 1e3) if rest else float("nan")
        out.append(f"{short:<60} {len(durs):>6} {sum(durs) / 1e6:>10.3f} "
                   f"{sum(durs) / len(durs) / 1e3:>10.2f} {k:>5} {avg_rest:>18.2f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--skip", action="append", default=[],
                    help="NAME=K: ignore the first K dispatches of kernels matching NAME")
    a = ap.parse_args(argv)
    skip = {}
    for s in a.skip:
        k, v = s.split("=")
        skip[k] = int(v)
    print(summarize(a.db, skip))
    return 0


if __name__ == "__main__":
    sys.exit(main())
