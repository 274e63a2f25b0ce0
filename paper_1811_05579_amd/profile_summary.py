"""Summarise a rocprofv3 kernel-trace database (run_results.db) as text:
per-kernel call count, total and average duration (the --stats view)."""
import sqlite3
import sys


def summarise(db_path):
    con = sqlite3.connect(db_path)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':70s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for name, n, tot, avg, mn, mx in rows:
        out.append(f"{name[:70]:70s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} "
                   f"{mx / 1e3:9.2f} {100 * tot / total:6.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1]))
