"""Summaries of rocprofv3 result databases (SQLite ``*_results.db``).

Measurement tooling; runs on any host, no GPU needed.

  python -m paper_2104_04347_amd.profsum trace DB
      per-kernel dispatch table (calls, total / mean / min / max duration,
      register counts, grid and workgroup sizes) from a --kernel-trace run

  python -m paper_2104_04347_amd.profsum trace DB --last K [--skip S]
      the same over each kernel's last K dispatches in launch order (the
      timed half-steps of a run, without its warm-up dispatches)

  python -m paper_2104_04347_amd.profsum counters DB
      per-kernel mean / min / max of every counter of a --pmc run

  python -m paper_2104_04347_amd.profsum insts DB --kernel SUBSTR --key NAME --N N
          [--sources 1d|2d] [--dispatches A:B] [--out profiles/valu_insts.json]
      mean SQ_INSTS_VALU (64-lane VALU instructions) per dispatch of the
      kernel whose name contains SUBSTR, from a --pmc run, keyed by NAME and
      stamped with the kernel sources' hash like the traffic record

  python -m paper_2104_04347_amd.profsum traffic FETCH_DB WRITE_DB --kernel SUBSTR
          --key NAME --N N --copy-mib M [--sources 1d|2d] [--dispatches A:B] [--out profiles/traffic.json]
      HBM bytes per dispatch of the kernel whose name contains SUBSTR, from a
      FETCH_SIZE run and a WRITE_SIZE run (both in KiB per dispatch), each
      scaled by what the same counter reads for the runtime's device-to-device
      copy of M MiB profiled in the same run (the largest copy dispatch).  The
      record is keyed by NAME and stamped with the SHA-256 of the kernel
      sources' code (the 1D, the 1D two-cells-per-lane or the 2D half-step's,
      comments removed: --sources 1d | 1d_wide | 2d), so that
      a later kernel change invalidates it.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


# the sources the single-instance 1D half-step kernel is compiled from, and
# those of the 2D half-step kernels
KERNEL_SOURCES = ("wcc_cell.hpp", "wcc_internal.hpp", "wcc_kernels.hip", "wcc_tile.hpp", "wcc_rn.hpp")
KERNEL_SOURCES_2D = ("wcc2d_cell.hpp", "wcc2d_internal.hpp", "wcc2d_kernels.hip", "wcc_internal.hpp", "wcc_tile.hpp",
                     "wcc_rn.hpp")
# the 1D kernel with two old cells per lane (launch variant 4)
KERNEL_SOURCES_WIDE = ("wcc_cell.hpp", "wcc_internal.hpp", "wcc_kernels_wide.hip", "wcc_tile.hpp", "wcc_wide.hpp",
                       "wcc_rn.hpp")
SOURCE_SETS = {"1d": KERNEL_SOURCES, "2d": KERNEL_SOURCES_2D, "1d_wide": KERNEL_SOURCES_WIDE}


def code_only(text: str) -> str:
    """C++ source without comments and blank lines, runs of blanks within a
    line made one (string literals in these sources hold no comment markers
    and no runs of blanks)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(" ".join(line.split()) for line in text.splitlines() if line.strip())


def kernel_source_hash(sources: str = "1d", read=None) -> str:
    """SHA-256 over the code (comments removed) of the sources of the 1D (or
    2D) half-step kernel.  `read(name)` supplies a file's text (default: the
    working tree)."""
    if read is None:
        def read(name):
            with open(os.path.join(CSRC, name)) as f:
                return f.read()
    h = hashlib.sha256()
    for name in SOURCE_SETS[sources]:
        h.update(name.encode() + b"\0" + code_only(read(name)).encode())
    return h.hexdigest()


def trace_table(db: str, last: int = 0, skip: int = 0) -> str:
    con = sqlite3.connect(db)
    if last > 0:
        # each kernel's last `last` dispatches (launch order = start time),
        # before its last `skip` ones
        con.execute(f"""create temp view sel as select * from (select *, row_number() over
                        (partition by name order by start desc) as rn from kernels)
                        where rn > {int(skip)} and rn <= {int(skip) + int(last)}""")
        table = "sel"
    else:
        table = "kernels"
    rows = con.execute(f"""select name, count(*), sum(duration), avg(duration), min(duration), max(duration),
                          max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(grid_x), max(workgroup_x)
                          from {table} group by name order by sum(duration) desc""").fetchall()
    tot = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':72s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
           f"{'%':>6s} vgpr agpr sgpr grid wg"]
    for r in rows:
        out.append(f"{r[0][:72]:72s} {r[1]:6d} {r[2] / 1e3:10.1f} {r[3] / 1e3:9.2f} {r[4] / 1e3:9.2f} "
                   f"{r[5] / 1e3:9.2f} {100 * r[2] / tot:6.2f} {r[6]} {r[7]} {r[8]} {r[9]} {r[10]}")
    return "\n".join(out)


def counter_values(db: str) -> dict:
    """{kernel name: {counter: [value per dispatch]}}"""
    con = sqlite3.connect(db)
    agg: dict = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, counter, value in con.execute("select kernel_name, counter_name, value from counters_collection "
                                            "order by dispatch_id"):
        agg[name][counter].append(float(value))
    return agg


def counters_table(db: str) -> str:
    out = []
    for k, d in counter_values(db).items():
        out.append(k[:100])
        for cn, v in sorted(d.items()):
            out.append(f"   {cn:28s} n={len(v):5d} mean={statistics.fmean(v):.6g} min={min(v):.6g} max={max(v):.6g}")
    return "\n".join(out)


def _one(db: str, counter: str, match: str, select: slice = slice(None)):
    agg = counter_values(db)
    ks = [k for k in agg if match in k]
    if len(ks) != 1:
        raise SystemExit(f"{db}: {len(ks)} kernels match {match!r}: {ks}")
    vals = (agg[ks[0]].get(counter) or [])[select]
    if not vals:
        raise SystemExit(f"{db}: no {counter} values for {ks[0]}")
    copies = agg.get(COPY_KERNEL, {}).get(counter)
    if not copies:
        raise SystemExit(f"{db}: no {counter} values for the calibration copy {COPY_KERNEL}")
    return ks[0], vals, max(copies)


def traffic(fetch_db: str, write_db: str, match: str, key: str, N: int, copy_mib: int, out: str | None,
            sources: str = "1d", select: slice = slice(None)) -> dict:
    name, fv, fcopy = _one(fetch_db, "FETCH_SIZE", match, select)
    _, wv, wcopy = _one(write_db, "WRITE_SIZE", match, select)
    copy_kib = copy_mib * 1024.0
    ff, wf = copy_kib / fcopy, copy_kib / wcopy
    rec = {
        "kernel_name": name,
        "source_sha256": kernel_source_hash(sources),
        "sources": sources,
        "N": N,
        "dispatches": [len(fv), len(wv)],
        "fetch_kib_raw_mean": statistics.fmean(fv),
        "write_kib_raw_mean": statistics.fmean(wv),
        "copy_mib": copy_mib,
        "copy_fetch_kib_raw": fcopy,
        "copy_write_kib_raw": wcopy,
        "fetch_factor": ff,
        "write_factor": wf,
        "fetch_bytes": statistics.fmean(fv) * 1024.0 * ff,
        "write_bytes": statistics.fmean(wv) * 1024.0 * wf,
    }
    if out:
        try:
            with open(out) as f:
                allrec = json.load(f)
        except (OSError, ValueError):
            allrec = {}
        allrec[key] = rec
        with open(out, "w") as f:
            json.dump(allrec, f, indent=1, sort_keys=True)
            f.write("\n")
    return rec


def insts(db: str, match: str, key: str, N: int, out: str | None, sources: str = "1d",
          select: slice = slice(None)) -> dict:
    agg = counter_values(db)
    ks = [k for k in agg if match in k]
    if len(ks) != 1:
        raise SystemExit(f"{db}: {len(ks)} kernels match {match!r}: {ks}")
    vals = (agg[ks[0]].get("SQ_INSTS_VALU") or [])[select]
    if not vals:
        raise SystemExit(f"{db}: no SQ_INSTS_VALU values for {ks[0]}")
    waves = (agg[ks[0]].get("SQ_WAVES") or [])[select]
    rec = {"kernel_name": ks[0], "source_sha256": kernel_source_hash(sources), "sources": sources, "N": N,
           "dispatches": len(vals), "sq_insts_valu": statistics.fmean(vals),
           "sq_insts_valu_min": min(vals), "sq_insts_valu_max": max(vals)}
    if waves:
        rec["sq_waves"] = statistics.fmean(waves)
    if out:
        try:
            with open(out) as f:
                allrec = json.load(f)
        except (OSError, ValueError):
            allrec = {}
        allrec[key] = rec
        with open(out, "w") as f:
            json.dump(allrec, f, indent=1, sort_keys=True)
            f.write("\n")
    return rec


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--last", type=int, default=0, help="only each kernel's last K dispatches")
    t.add_argument("--skip", type=int, default=0, help="with --last: the K dispatches before each kernel's last S")
    i = sub.add_parser("insts")
    i.add_argument("db")
    i.add_argument("--kernel", required=True)
    i.add_argument("--key", required=True)
    i.add_argument("--N", type=int, required=True)
    i.add_argument("--sources", choices=tuple(SOURCE_SETS), default="1d")
    i.add_argument("--dispatches", default=":")
    i.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("db")
    r = sub.add_parser("traffic")
    r.add_argument("fetch_db")
    r.add_argument("write_db")
    r.add_argument("--kernel", required=True)
    r.add_argument("--key", required=True)
    r.add_argument("--N", type=int, required=True)
    r.add_argument("--copy-mib", type=int, required=True)
    r.add_argument("--sources", choices=tuple(SOURCE_SETS), default="1d")
    r.add_argument("--dispatches", default=":",
                   help="A:B, the kernel's dispatches A to B-1 in launch order (a kernel run by several legs)")
    r.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.db, a.last, a.skip))
    elif a.cmd == "counters":
        print(counters_table(a.db))
    elif a.cmd == "insts":
        lo, hi = (int(v) if v else None for v in a.dispatches.split(":"))
        json.dump(insts(a.db, a.kernel, a.key, a.N, a.out, a.sources, slice(lo, hi)), sys.stdout, indent=1)
        print()
    else:
        lo, hi = (int(v) if v else None for v in a.dispatches.split(":"))
        json.dump(traffic(a.fetch_db, a.write_db, a.kernel, a.key, a.N, a.copy_mib, a.out, a.sources, slice(lo, hi)),
                  sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
