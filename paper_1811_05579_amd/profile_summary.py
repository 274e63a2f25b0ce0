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
  python3 profile_summary.py --pmc-steps FETCH_CSV WRITE_CSV FETCH_SCALE WRITE_SCALE MARK FROM TO [PER]
      HBM bytes per step from one FETCH_SIZE and one WRITE_SIZE run of the same
      program: every dispatch (all kernels) from the FROM-th to before the TO-th
      dispatch of the kernel whose name contains MARK (0-based; TO past the last
      one: to the end of the run), KiB x 1024 x the copy-calibrated scale,
      summed per kernel and divided by the steps, (TO - FROM) / PER for PER
      dispatches of MARK per step (default 1).
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


def _short(name):
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(", 1)[0]


def summarise_pmc_steps(fetch_csv, write_csv, fetch_scale, write_scale, mark, first, last, per_step=1):
    steps = (last - first) / per_step
    out = []
    per = {}
    totals = {}
    for counter, path, scale in (("FETCH_SIZE", fetch_csv, fetch_scale), ("WRITE_SIZE", write_csv, write_scale)):
        rows = {}
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                d = int(row["Dispatch_Id"])
                if d not in rows:
                    rows[d] = [row["Kernel_Name"], 0.0]
                rows[d][1] += float(row["Counter_Value"])
        marks = sorted(d for d, (k, _) in rows.items() if mark in k)
        lo, hi = marks[first], (marks[last] if last < len(marks) else max(rows) + 1)
        tot = 0.0
        for d, (k, v) in rows.items():
            if lo <= d < hi:
                b = v * 1024.0 * scale / steps
                per.setdefault(_short(k), [0.0, 0.0])[0 if counter == "FETCH_SIZE" else 1] += b
                tot += b
        totals[counter] = tot
    out.append(f"{'kernel':44s} {'read B/step':>12s} {'write B/step':>12s} {'total':>12s}")
    for k, (r, w) in sorted(per.items(), key=lambda kv: -(kv[1][0] + kv[1][1])):
        out.append(f"{k[:44]:44s} {r:12.4e} {w:12.4e} {r + w:12.4e}")
    out.append(f"{'per step':44s} {totals['FETCH_SIZE']:12.4e} {totals['WRITE_SIZE']:12.4e} "
               f"{totals['FETCH_SIZE'] + totals['WRITE_SIZE']:12.4e}  ({steps} steps)")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] in ("-h", "--help"):
        print(__doc__)
    elif sys.argv[1] == "--window":
        print(summarise_window(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5])))
    elif len(sys.argv) >= 2 and sys.argv[1] == "--launches":
        print(summarise_launches(sys.argv[2], sys.argv[3], float(sys.argv[4])))
    elif sys.argv[1] == "--pmc-steps":
        print(summarise_pmc_steps(sys.argv[2], sys.argv[3], float(sys.argv[4]), float(sys.argv[5]), sys.argv[6],
                                  int(sys.argv[7]), int(sys.argv[8]), int(sys.argv[9]) if len(sys.argv) > 9 else 1))
    elif len(sys.argv) >= 2 and sys.argv[1] == "--pmc":
        print(summarise_pmc(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) > 4 else None))
    else:
        print(summarise(sys.argv[1]))
