"""Summarise a rocprofv3 SQLite output (rocpd): per-kernel calls, total and
average duration, and, for one kernel, the launches at a given grid size.

usage: python profiles/summarize_rocpd.py RESULTS.db [KERNEL_SUBSTRING GRID_X]"""
import sqlite3
import sys


def main():
    con = sqlite3.connect(sys.argv[1])
    cur = con.cursor()
    rows = cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    # top_kernels reports microseconds; the kernels table reports nanoseconds
    print(f"{'kernel':60s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}")
    for name, calls, tot, avg, pct in rows[:20]:
        short = name.split("(")[0].replace("void ", "")
        print(f"{short[:60]:60s} {calls:8d} {tot / 1e3:10.2f} {avg:9.2f} {pct:6.2f}")
    if len(sys.argv) > 3:
        sub, gx = sys.argv[2], int(sys.argv[3])
        r = cur.execute("select count(*), avg(duration), min(duration), max(duration) from kernels "
                        "where name like ? and grid_x = ?", (f"%{sub}%", gx)).fetchone()
        print(f"\n{sub} launches with grid_x={gx}: count={r[0]} avg_us={r[1] / 1e3:.2f} "
              f"min_us={r[2] / 1e3:.2f} max_us={r[3] / 1e3:.2f}")


if __name__ == "__main__":
    main()
