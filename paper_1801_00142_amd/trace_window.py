"""Per-kernel statistics of a rocprofv3 kernel trace inside a time window.

    python -m paper_1801_00142_amd.trace_window TRACE.csv START_NS END_NS [TOP]

TRACE.csv is the kernel trace of `rocprofv3 --kernel-trace -f csv`; the
window is given on the tracer's clock (CLOCK_BOOTTIME nanoseconds, which
bench.py reports around its timed steps as `timed_window_ns`).  Prints, for
the TOP kernels by total duration, the dispatches that start and end inside
the window: calls, total and average duration.  The trace is read as a
stream (kernel traces of a full bench run hold millions of dispatches).
"""
import csv
import sys
from collections import defaultdict


def window_stats(path: str, start: int, end: int):
    calls = defaultdict(int)
    total = defaultdict(int)
    seen = 0
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            seen += 1
            if seen % 2_000_000 == 0:
                print(f"# {seen} dispatches read", file=sys.stderr, flush=True)
            a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            if a >= start and b <= end:
                name = row["Kernel_Name"]
                calls[name] += 1
                total[name] += b - a
    return calls, total, seen


def main():
    if len(sys.argv) < 4:
        print(__doc__)
        sys.exit(2)
    path, start, end = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    top = int(sys.argv[4]) if len(sys.argv) > 4 else 16
    calls, total, seen = window_stats(path, start, end)
    busy = sum(total.values())
    print(f"window {start} .. {end} ns ({(end - start) / 1e9:.3f} s): {sum(calls.values())} of {seen} dispatches, "
          f"kernel time {busy / 1e9:.3f} s")
    print("Name\tCalls\tTotalNs\tAverageNs\tPercent")
    for name in sorted(total, key=total.get, reverse=True)[:top]:
        short = name if len(name) <= 110 else name[:107] + "..."
        print(f"{short}\t{calls[name]}\t{total[name]}\t{total[name] / calls[name]:.1f}\t"
              f"{100.0 * total[name] / busy:.2f}")


if __name__ == "__main__":
    main()
