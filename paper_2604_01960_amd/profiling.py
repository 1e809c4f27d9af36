"""Summaries of rocprofv3 results (the SQLite database it writes with
``-d DIR -o NAME``), for the per-kernel tables and HBM traffic figures that
sit under ``profiles/``.

    python -m paper_2604_01960_amd.profiling stats DB [--regex R]
        per-kernel table (calls, average / min / max duration) of a
        ``--kernel-trace`` run, grouped by kernel name and grid
    python -m paper_2604_01960_amd.profiling counter DB COUNTER --regex R
        mean per-dispatch value of one ``--pmc`` counter over the matching
        kernels
    python -m paper_2604_01960_amd.profiling traffic --fetch DB --write DB \\
        --cal-fetch DB --cal-write DB --cal-bytes N --regex R --cal-regex R \\
        --source FILE [--source FILE ...] --command CMD --out FILE.md
        HBM bytes per dispatch of the matching kernel: FETCH_SIZE and
        WRITE_SIZE (KiB per dispatch) scaled by the ratio of the bytes a plain
        copy kernel of known size moves to what the same counters read for it.
        The result carries the SHA-256 of the kernel's sources, so a reader
        can tell when the kernel has changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import re
import sqlite3
import sys
from typing import Dict, List, Tuple

TRAFFIC_TAG = "traffic-json:"


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def kernel_stats(db: str, regex: str = "", by_name: bool = False, since: str = "") -> List[Tuple]:
    """(name, blocks, block size, LDS bytes, VGPRs, calls, avg us, min us, max us,
    total ms), by total time.  by_name: one row per kernel (grid and LDS given as
    their range over the dispatches).  since: only the dispatches that start at
    or after the first dispatch of a kernel matching this pattern (to leave
    out an index build that runs before the searches)."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x, grid_y, workgroup_x, duration, lds_size, vgpr_count, start from kernels "
                     "order by start").fetchall()
    if since:
        sx = re.compile(since)
        first = next((r[7] for r in rows if sx.search(_short(r[0]))), None)
        rows = [] if first is None else [r for r in rows if r[7] >= first]
    g: Dict[Tuple, List[Tuple]] = collections.defaultdict(list)
    rx = re.compile(regex) if regex else None
    for name, gx, gy, wx, dur, lds, vg, _ in rows:
        short = _short(name)
        if rx and not rx.search(short):
            continue
        key = (short, wx, vg) if by_name else (short, gx // max(1, wx), gy, wx, lds, vg)
        g[key].append((dur / 1000.0, gx // max(1, wx), gy, lds))
    out = []
    for key, recs in sorted(g.items(), key=lambda kv: -sum(r[0] for r in kv[1])):
        ds = [r[0] for r in recs]
        if by_name:
            name, wx, vg = key
            bx = sorted({r[1] for r in recs})
            by = sorted({r[2] for r in recs})
            ld = sorted({r[3] for r in recs})
            span = lambda v: str(v[0]) if len(v) == 1 else f"{v[0]}-{v[-1]}"
            grid, lds = f"{span(bx)},{span(by)}", span(ld)
        else:
            name, bx, by, wx, lds, vg = key
            grid = f"{bx},{by}"
        out.append((name, grid, wx, lds, vg, len(ds), sum(ds) / len(ds), min(ds), max(ds), sum(ds) / 1000.0))
    return out


def stats_markdown(db: str, regex: str = "", by_name: bool = False, since: str = "") -> str:
    lines = ["| kernel | grid (blocks) | block | LDS B | VGPR | calls | avg us | min us | max us | total ms |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for name, grid, wx, lds, vg, n, avg, mn, mx, tot in kernel_stats(db, regex, by_name, since):
        lines.append(f"| `{name}` | {grid} | {wx} | {lds} | {vg} | {n} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {tot:.1f} |")
    return "\n".join(lines)


def counter_per_dispatch(db: str, counter: str, regex: str) -> Tuple[float, int]:
    """Mean over the matching dispatches of the counter's per-dispatch total
    (the counter's values summed over its instances), and the dispatch count."""
    c = sqlite3.connect(db)
    rx = re.compile(regex)
    per: Dict[int, float] = collections.defaultdict(float)
    for name, disp, cname, val in c.execute(
            "select kernel_name, dispatch_id, counter_name, value from counters_collection"):
        if cname != counter or not rx.search(_short(name)):
            continue
        per[disp] += float(val)
    if not per:
        raise SystemExit(f"no dispatch of /{regex}/ with counter {counter} in {db}")
    return sum(per.values()) / len(per), len(per)


def counter_by_grid(db: str, counter: str, regex: str) -> List[Tuple]:
    """Per grid shape of the matching dispatches: (grid, dispatches, mean of
    the counter's per-dispatch total).  The grid columns are taken from the
    counter table when it has them."""
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)").fetchall()]
    gcols = [x for x in ("grid_size_x", "grid_size_y", "grid_size", "workgroup_size") if x in cols]
    sel = ", ".join(["kernel_name", "dispatch_id", "counter_name", "value"] + gcols)
    rx = re.compile(regex)
    per: Dict[int, float] = collections.defaultdict(float)
    grid: Dict[int, Tuple] = {}
    for row in c.execute(f"select {sel} from counters_collection"):
        name, disp, cname, val = row[:4]
        if cname != counter or not rx.search(_short(name)):
            continue
        per[disp] += float(val)
        grid[disp] = tuple(row[4:])
    g: Dict[Tuple, List[float]] = collections.defaultdict(list)
    for d, v in per.items():
        g[grid[d]].append(v)
    return [(k, len(v), sum(v) / len(v)) for k, v in sorted(g.items())]


def sources_sha256(paths: List[str]) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic(md_path: str) -> dict:
    """The traffic record written by ``traffic`` (the line tagged TRAFFIC_TAG)."""
    with open(md_path) as f:
        for line in f:
            line = line.strip().strip("`")
            if line.startswith(TRAFFIC_TAG):
                return json.loads(line[len(TRAFFIC_TAG):])
    raise ValueError(f"no traffic record in {md_path}")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2604_01960_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--regex", default="")
    s.add_argument("--by-name", action="store_true", help="one row per kernel name")
    s.add_argument("--since", default="", help="only dispatches from the first one of a kernel matching this")
    c = sub.add_parser("counter")
    c.add_argument("db")
    c.add_argument("counter")
    c.add_argument("--regex", required=True)
    c.add_argument("--by-grid", action="store_true", help="one line per grid shape")
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--cal-fetch", "--cal-write", "--regex", "--cal-regex", "--out", "--command"):
        t.add_argument(a, required=True)
    t.add_argument("--cal-bytes", type=int, required=True, help="bytes the calibration copy reads (= writes)")
    t.add_argument("--source", action="append", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_markdown(args.db, args.regex, args.by_name, args.since))
    elif args.cmd == "counter" and args.by_grid:
        for grid, n, v in counter_by_grid(args.db, args.counter, args.regex):
            print(f"{args.counter} grid {grid}: {v:.1f} per dispatch over {n} dispatches")
    elif args.cmd == "counter":
        v, n = counter_per_dispatch(args.db, args.counter, args.regex)
        print(f"{args.counter}: {v:.1f} per dispatch over {n} dispatches")
    else:
        f_kib, nf = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.regex)
        w_kib, nw = counter_per_dispatch(args.write, "WRITE_SIZE", args.regex)
        cf_kib, _ = counter_per_dispatch(args.cal_fetch, "FETCH_SIZE", args.cal_regex)
        cw_kib, _ = counter_per_dispatch(args.cal_write, "WRITE_SIZE", args.cal_regex)
        ffac = args.cal_bytes / (cf_kib * 1024.0)
        wfac = args.cal_bytes / (cw_kib * 1024.0)
        fetch = f_kib * 1024.0 * ffac
        write = w_kib * 1024.0 * wfac
        rec = {"kernel_regex": args.regex, "fetch_bytes": round(fetch), "write_bytes": round(write),
               "traffic_bytes": round(fetch + write), "dispatches": [nf, nw],
               "fetch_kib_raw": round(f_kib, 1), "write_kib_raw": round(w_kib, 1),
               "fetch_factor": round(ffac, 4), "write_factor": round(wfac, 4),
               "calibration_bytes": args.cal_bytes, "sources": args.source,
               "sources_sha256": sources_sha256(args.source)}
        md = [f"# HBM traffic per dispatch of `{args.regex}`", "",
              "Command (run from the repository root):", "", "```", args.command, "```", "",
              "| quantity | value |", "|---|---|",
              f"| FETCH_SIZE per dispatch (raw, KiB) | {f_kib:.1f} over {nf} dispatches |",
              f"| WRITE_SIZE per dispatch (raw, KiB) | {w_kib:.1f} over {nw} dispatches |",
              f"| copy calibration: bytes read = written | {args.cal_bytes} |",
              f"| copy calibration FETCH_SIZE / WRITE_SIZE (KiB) | {cf_kib:.1f} / {cw_kib:.1f} |",
              f"| scale factors fetch / write | {ffac:.4f} / {wfac:.4f} |",
              f"| HBM bytes fetched per dispatch | {fetch:.4g} |",
              f"| HBM bytes written per dispatch | {write:.4g} |",
              f"| traffic per dispatch | {fetch + write:.4g} |", "",
              f"`{TRAFFIC_TAG} {json.dumps(rec)}`", ""]
        with open(args.out, "w") as f:
            f.write("\n".join(md))
        print("\n".join(md))


if __name__ == "__main__":
    main(sys.argv[1:])
