"""Summarise rocprofv3 output as text.

  python3 profile_summary.py RUN_results.db
      kernel-trace database: per-kernel call count, total, average, min and
      max duration in microseconds (the --stats view).
  python3 profile_summary.py --pmc COUNTER_CSV KERNEL_SUBSTRING
      counter-collection CSV of one --pmc run: per-dispatch values of the
      counter (KiB for FETCH_SIZE / WRITE_SIZE) for the kernels whose name
      contains KERNEL_SUBSTRING: count, mean, min, max.
  python3 profile_summary.py --pmc COUNTER_CSV KERNEL_SUBSTRING MIN
      the same over the dispatches whose value is at least MIN (e.g. to leave
      out launches that returned at once because a solve had converged).
  python3 profile_summary.py --launches RUN_results.db KERNEL_SUBSTRING MIN_US
      count, mean, min, max duration of the matching kernel's launches that
      took at least MIN_US microseconds.
  python3 profile_summary.py --window RUN_results.db KERNEL_SUBSTRING FIRST COUNT
      durations of COUNT launches of the matching kernel, in launch order,
      starting at launch FIRST (negative: counted from the last launch), e.g.
      the timed steps of a run that ends with one extra step: -51 50.
"""
import csv
import sqlite3
import sys


def _open(db_path):
    # read-only: a mistyped path fails instead of creating an empty database
    return sqlite3.connect(f"file:{db_path}?mode=ro", uri=True)


def summarise(db_path):
    con = _open(db_path)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':70s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for name, n, tot, avg, mn, mx in rows:
        out.append(f"{name[:70]:70s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} "
                   f"{mx / 1e3:9.2f} {100 * tot / total:6.1f}")
    return "\n".join(out)


def summarise_window(db_path, kernel_substring, first, count):
    con = _open(db_path)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    d = [dur for name, dur in rows if kernel_substring in name]
    sel = d[first:first + count] if first + count != 0 else d[first:]
    if len(sel) != count:
        return f"only {len(sel)} of {count} '{kernel_substring}' launches from {first} ({len(d)} in all)"
    mean = sum(sel) / count
    return (f"'{kernel_substring}' launches {first}..{first + count - 1} of {len(d)} (launch order): "
            f"mean {mean / 1e3:.2f} us  min {min(sel) / 1e3:.2f}  max {max(sel) / 1e3:.2f}")


def summarise_launches(db_path, kernel_substring, min_us):
    con = _open(db_path)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    d = [dur / 1e3 for name, dur in rows if kernel_substring in name]
    sel = [x for x in d if x >= min_us]
    if not sel:
        return f"no '{kernel_substring}' launch of at least {min_us} us ({len(d)} in all)"
    return (f"'{kernel_substring}' launches >= {min_us} us: {len(sel)} of {len(d)}, mean {sum(sel) / len(sel):.2f} us  "
            f"min {min(sel):.2f}  max {max(sel):.2f}")


def counter_values(csv_path, kernel_substring):
    """{counter name: [value per dispatch]} for the matching kernels (rows of
    one dispatch are summed: some counters come per shader engine or XCD)."""
    per = {}
    with open(csv_path, newline="") as f:
        for row in csv.DictReader(f):
            if kernel_substring not in row["Kernel_Name"]:
                continue
            key = (row["Counter_Name"], row["Dispatch_Id"])
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, _), v in sorted(per.items(), key=lambda kv: int(kv[0][1])):
        out.setdefault(name, []).append(v)
    return out


def summarise_pmc(csv_path, kernel_substring, vmin=None):
    lines = []
    for name, vals in counter_values(csv_path, kernel_substring).items():
        if vmin is not None:
            vals = [v for v in vals if v >= vmin]
            if not vals:
                continue
        lines.append(f"{name} over {len(vals)} dispatches of '{kernel_substring}': mean {sum(vals) / len(vals):.1f} "
                     f"min {min(vals):.1f} max {max(vals):.1f}")
    return "\n".join(lines) if lines else f"no '{kernel_substring}' dispatches in {csv_path}"


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] in ("-h", "--help"):
        print(__doc__)
    elif sys.argv[1] == "--window":
        print(summarise_window(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5])))
    elif len(sys.argv) >= 2 and sys.argv[1] == "--launches":
        print(summarise_launches(sys.argv[2], sys.argv[3], float(sys.argv[4])))
    elif len(sys.argv) >= 2 and sys.argv[1] == "--pmc":
        print(summarise_pmc(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) > 4 else None))
    else:
        print(summarise(sys.argv[1]))
