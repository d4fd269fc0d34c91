"""Text summaries of rocprofv3 result databases (the `--kernel-trace --stats` and `--pmc`
runs behind the committed profile summaries).

    python3 -m paper_1602_00138_amd.rocsum DIR [--match REGEX] [--busy]

DIR is the rocprofv3 output directory (-d); the first *_results.db below it is read.
Prints the per-kernel time table (calls, total and average duration, share) and, for
counter runs, the per-kernel averages of every collected counter.  --match keeps kernels
whose name matches REGEX.  --busy also prints the GPU busy fraction: the union of all
kernel execution intervals over the span from the first kernel start to the last kernel
end (the share of wall time with at least one kernel running)."""
import argparse
import glob
import re
import sqlite3
import sys


def _db(path: str) -> sqlite3.Connection:
    dbs = sorted(glob.glob(path + "/**/*_results.db", recursive=True))
    if not dbs:
        sys.exit(f"no *_results.db under {path}")
    return sqlite3.connect(dbs[0])


def _tables(cur) -> set:
    return {r[0] for r in cur.execute("select name from sqlite_master where type in ('table','view')")}


def kernel_table(cur, match):
    rows = []
    for name, calls, total, avg, pct in cur.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        if match and not re.search(match, name):
            continue
        rows.append((name, calls, total, avg, pct))
    print("kernel | calls | total_us | avg_us | pct")
    for name, calls, total, avg, pct in rows:
        # top_kernels holds durations in microseconds
        print(f"{name[:160]} | {calls} | {total:.1f} | {avg:.3f} | {pct:.2f}")


def busy_fraction(cur):
    iv = sorted(cur.execute("select start, end from kernels"))
    if not iv:
        return
    busy, cs, ce = 0, iv[0][0], iv[0][1]
    for s, e in iv[1:]:
        if s > ce:
            busy += ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    busy += ce - cs
    span = max(e for _, e in iv) - iv[0][0]
    print(f"busy: {busy / 1e6:.1f} ms of kernels over a {span / 1e6:.1f} ms span = "
          f"{busy / span:.3f}")


def counter_table(cur, match):
    q = ("select kernel_name, counter_name, count(*), avg(value) from counters_collection "
         "group by kernel_name, counter_name")
    try:
        rows = list(cur.execute(q))
    except sqlite3.Error:
        return
    print("kernel | counter | dispatches | average per dispatch")
    for name, cname, n, avg in sorted(rows, key=lambda r: -r[2] * r[3]):
        if match and not re.search(match, name):
            continue
        print(f"{name[:160]} | {cname} | {n} | {avg:.1f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--match", default=None)
    ap.add_argument("--busy", action="store_true")
    a = ap.parse_args()
    con = _db(a.dir)
    cur = con.cursor()
    t = _tables(cur)
    if "top_kernels" in t:
        kernel_table(cur, a.match)
    if a.busy and "kernels" in t:
        busy_fraction(cur)
    if "counters_collection" in t:
        counter_table(cur, a.match)


if __name__ == "__main__":
    main()
