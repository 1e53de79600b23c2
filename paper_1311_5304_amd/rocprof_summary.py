"""Summarise rocprofv3 result databases (SQLite) per kernel.

    python -m paper_1311_5304_amd.rocprof_summary DB [DB ...]

For kernel-trace databases it prints, per kernel, the dispatch count and the
average / min / max duration.  For counter databases (--pmc) it prints, per
kernel and counter, the average value per dispatch.
"""
from __future__ import annotations

import collections
import sqlite3
import sys


def _short(name: str, width: int = 72) -> str:
    return name if len(name) <= width else name[:width - 3] + "..."


def kernel_durations(db_path: str):
    db = sqlite3.connect(db_path)
    out = collections.defaultdict(list)
    try:
        for name, dur in db.execute("select name, duration from kernels"):
            out[name].append(dur)
    except sqlite3.OperationalError:
        pass
    return out


def counters(db_path: str):
    """-> {kernel: {counter: [value per dispatch]}} (values summed over instances)."""
    db = sqlite3.connect(db_path)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    try:
        rows = db.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection")
        for disp, kname, cname, value in rows:
            per[(disp, kname)][cname] += value
            names[disp] = kname
    except sqlite3.OperationalError:
        return {}
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for (disp, kname), cs in per.items():
        for cname, v in cs.items():
            out[kname][cname].append(v)
    return out


def main(argv):
    for path in argv:
        print(f"== {path}")
        for name, d in sorted(kernel_durations(path).items(), key=lambda kv: -sum(kv[1])):
            print(f"  {_short(name):72s} n={len(d):5d} avg={sum(d) / len(d) / 1e3:9.3f} us "
                  f"min={min(d) / 1e3:9.3f} max={max(d) / 1e3:9.3f}")
        for kname, cs in counters(path).items():
            for cname, vals in sorted(cs.items()):
                print(f"  {_short(kname):72s} {cname:28s} avg/dispatch={sum(vals) / len(vals):.6g} (n={len(vals)})")


if __name__ == "__main__":
    main(sys.argv[1:])
