"""Summaries of rocprofv3 result databases (rocpd SQLite).

  python -m paper_2502_11385_amd.rocprof_summary stats DB
      per-kernel calls / total / average duration (kernel-trace run)
  python -m paper_2502_11385_amd.rocprof_summary counters DB --kernel NAME \
        [--json OUT --source FILES...]
      per-counter averages per dispatch (and per wave with SQ_WAVES) of one
      kernel in a --pmc run
  python -m paper_2502_11385_amd.rocprof_summary traffic FETCH_DB WRITE_DB \
        --kernel tile_kernel --copy-bytes 1073741824 [--json OUT]
      HBM bytes per dispatch of one kernel from FETCH_SIZE and WRITE_SIZE
      runs, each scaled by what the same counter reads for a device copy of
      known size in the same run (read = write = copy-bytes)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys


def sources_hash(paths) -> str:
    """First 16 hex digits of the SHA-256 over the files' bytes, in order."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(db: str, sql: str):
    c = sqlite3.connect(db)
    try:
        return c.execute(sql).fetchall()
    finally:
        c.close()


def kernel_stats(db: str):
    """[(name, calls, total_us, avg_us)] sorted by total time."""
    rows = _rows(db, "select name, count(*), sum(duration), avg(duration) "
                     "from kernels group by name order by sum(duration) desc")
    return [(n, int(c), t / 1e3, a / 1e3) for n, c, t, a in rows]


def counter_per_dispatch(db: str, counter: str):
    """{dispatch_id: (kernel_name, value)} for one counter (summed over
    its components)."""
    rows = _rows(db, "select dispatch_id, kernel_name, sum(value) from "
                     "counters_collection where counter_name = '%s' "
                     "group by dispatch_id" % counter)
    return {d: (k, v) for d, k, v in rows}


def _copy_value(vals: dict, copy_bytes: int) -> float:
    """Counter value of the calibration copy: the dispatch whose name marks a
    copy and whose value is largest (the 1 GiB copy dominates any other)."""
    best = None
    for k, v in vals.values():
        if "copy" in k.lower() or "elementwise" in k.lower():
            if best is None or v > best:
                best = v
    if best is None:
        raise RuntimeError("no copy kernel found in the counter run")
    return float(best)


def traffic(fetch_db: str, write_db: str, kernel: str, copy_bytes: int):
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")
    fc, wc = _copy_value(f, copy_bytes), _copy_value(w, copy_bytes)
    f_scale, w_scale = copy_bytes / fc, copy_bytes / wc
    fk = [v for k, v in f.values() if kernel in k]
    wk = [v for k, v in w.values() if kernel in k]
    if not fk or not wk:
        raise RuntimeError(f"kernel {kernel!r} not in counter runs")
    rd = sum(fk) / len(fk) * f_scale
    wr = sum(wk) / len(wk) * w_scale
    return {"kernel": kernel, "dispatches": [len(fk), len(wk)],
            "fetch_counter_avg": sum(fk) / len(fk),
            "write_counter_avg": sum(wk) / len(wk),
            "copy_fetch_counter": fc, "copy_write_counter": wc,
            "copy_bytes": copy_bytes,
            "fetch_scale_bytes_per_unit": f_scale,
            "write_scale_bytes_per_unit": w_scale,
            "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
            "bytes_per_launch": rd + wr}


def counters(db: str, kernel: str):
    """Per counter of a --pmc run: dispatches of `kernel`, average value per
    dispatch and, when SQ_WAVES was collected, the average per wave."""
    names = [r[0] for r in _rows(db, "select distinct counter_name from "
                                      "counters_collection")]
    per = {c: [v for k, v in counter_per_dispatch(db, c).values()
               if kernel in k] for c in names}
    waves = per.get("SQ_WAVES")
    out = []
    for c in sorted(names):
        vals = per[c]
        if not vals:
            continue
        avg = sum(vals) / len(vals)
        pw = (avg / (sum(waves) / len(waves))) if waves else None
        out.append((c, len(vals), avg, pw))
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", default="tile_kernel")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--json", default=None)
    t.add_argument("--source", default=None, nargs="+",
                   help="kernel source files whose combined hash is recorded")
    t.add_argument("--strategy", default="tiled")
    k = sub.add_parser("counters")
    k.add_argument("db")
    k.add_argument("--kernel", default="tile_kernel")
    k.add_argument("--json", default=None)
    k.add_argument("--source", default=None, nargs="+",
                   help="kernel source files whose combined hash is recorded")
    k.add_argument("--strategy", default="tiled")
    a = ap.parse_args()
    if a.cmd == "counters":
        rows = counters(a.db, a.kernel)
        print(f"{'counter':24s} {'dispatches':>10} {'avg/dispatch':>16} "
              f"{'avg/wave':>12}")
        for c, nd, avg, pw in rows:
            pws = f"{pw:12.2f}" if pw is not None else f"{'':>12}"
            print(f"{c:24s} {nd:10d} {avg:16.1f} {pws}")
        if a.json:
            r = {"kernel": a.kernel,
                 "per_dispatch": {c: avg for c, _, avg, _ in rows},
                 "dispatches": max((nd for _, nd, _, _ in rows), default=0)}
            if a.source:
                r["kernel_source_sha256_16"] = sources_hash(a.source)
                r["strategy"] = a.strategy
            with open(a.json, "w") as f:
                json.dump(r, f, indent=1)
        return 0
    if a.cmd == "stats":
        print(f"{'calls':>6} {'total_ms':>10} {'avg_us':>10}  kernel")
        for n, c, tot, avg in kernel_stats(a.db):
            print(f"{c:6d} {tot / 1e3:10.3f} {avg:10.1f}  {n[:110]}")
        return 0
    r = traffic(a.fetch_db, a.write_db, a.kernel, a.copy_bytes)
    if a.source:
        r["kernel_source_sha256_16"] = sources_hash(a.source)
        r["strategy"] = a.strategy
    print(json.dumps(r, indent=1))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(r, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
