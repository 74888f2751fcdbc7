"""Summarise a rocprofv3 kernel-trace database (``*_results.db``) as text:
per-kernel call count, total and average duration.  Used to write the short
summaries kept under profiles/."""
from __future__ import annotations

import sqlite3
import sys


def kernel_stats(db_path: str, limit: int = 20):
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels limit ?", (limit,)).fetchall()
    con.close()
    return rows


def main(argv):
    for path in argv[1:]:
        print(f"# {path}")
        print("| kernel | calls | total us | avg us | % |")
        print("|---|---|---|---|---|")
        for name, calls, total, avg, pct in kernel_stats(path):
            short = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            print(f"| {short} | {calls} | {total:.1f} | {avg:.2f} | {pct:.1f} |")


if __name__ == "__main__":
    main(sys.argv)
