"""Summarise a rocprofv3 kernel-trace database into a per-kernel table.

usage: python profiles/summarize.py <run_results.db> [title]
"""
import sqlite3
import sys


def main(db_path, title=""):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, count(*), sum(end-start), avg(end-start), min(end-start), max(end-start) "
                      "from kernels group by name order by sum(end-start) desc").fetchall()
    total = sum(r[2] for r in rows)
    print(f"# {title}\n")
    print("| kernel | calls | total ms | avg us | min us | max us | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for name, n, tot, avg, mn, mx in rows:
        short = name.split("(")[0]
        print(f"| {short} | {n} | {tot/1e6:.3f} | {avg/1e3:.2f} | {mn/1e3:.2f} | {mx/1e3:.2f} | {100*tot/total:.1f} |")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else "")
