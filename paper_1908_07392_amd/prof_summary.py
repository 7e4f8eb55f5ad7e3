"""Summarise a rocprofv3 results database (kernel trace) as a text table.

usage: python paper_1908_07392_amd/prof_summary.py <results.db> [command-line-that-produced-it]
"""
import sqlite3
import sys


def main():
    db = sys.argv[1]
    cmd = " ".join(sys.argv[2:])
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = []
    if cmd:
        out.append(f"command: {cmd}")
    # top_kernels reports durations in microseconds
    out.append(f"{'kernel':80s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'pct':>6s}")
    for name, calls, tot, avg, pct in rows:
        short = name if len(name) <= 80 else name[:77] + "..."
        out.append(f"{short:80s} {calls:6d} {tot:12.1f} {avg:10.2f} {pct:6.2f}")
    print("\n".join(out))


if __name__ == "__main__":
    main()
