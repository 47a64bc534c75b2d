"""Short text summaries of rocprofv3 output, per kernel.

  trace: python -m paper_1901_07374_amd.rocprof_summary trace RESULTS.db \
             --command "..." [--bench-json FILE]
         kernel calls, mean/min/max duration and share of GPU time from a
         --kernel-trace --stats run.
  pmc:   python -m paper_1901_07374_amd.rocprof_summary pmc FETCH.db WRITE.db \
             --copy-bytes B --command "..." --command "..."
         FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel, scaled by
         what the same counters read for a device copy of B bytes, written as
         `key = value` lines (HBM bytes per launch per kernel).
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3
import sys


def short_name(name: str) -> str:
    """'void tlsph::k_pass_b_staged<double>(tlsph::DevState, int)' ->
    'k_pass_b_staged<double>'."""
    s = name.strip()
    if s.startswith("void "):
        s = s[5:]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            s = s[:i]
            break
    s = s.replace("tlsph::", "")
    return re.sub(r"\s+", " ", s)


def _tables(c):
    return [r[0] for r in c.execute("select name from sqlite_master where type in ('table','view')")]


def _cols(c, t):
    return [r[1] for r in c.execute(f"pragma table_info('{t}')")]


def dispatch_durations(db: str):
    """{kernel: [duration ns, ...]} from the per-dispatch kernel view."""
    c = sqlite3.connect(db)
    tabs = _tables(c)
    for t in ("kernels", "kernel_dispatch", "rocpd_kernel_dispatch"):
        if t not in tabs:
            continue
        cols = _cols(c, t)
        name = next((k for k in ("name", "kernel_name") if k in cols), None)
        beg = next((k for k in ("start", "start_ns", "begin") if k in cols), None)
        end = next((k for k in ("end", "end_ns", "stop") if k in cols), None)
        if name and beg and end:
            out = collections.defaultdict(list)
            for n, b, e in c.execute(f'select "{name}", "{beg}", "{end}" from "{t}"'):
                out[short_name(str(n))].append(float(e) - float(b))
            return out
    if "top_kernels" in tabs:
        # aggregate view only: mean duration repeated per call
        cols = _cols(c, "top_kernels")
        print(f"# per-dispatch view missing; top_kernels columns {cols}", file=sys.stderr)
        out = {}
        for n, calls, avg in c.execute("select name, total_calls, average from top_kernels"):
            out[short_name(str(n))] = [float(avg)] * int(calls)
        return out
    raise SystemExit(f"{db}: no kernel table among {tabs}")


def trace(args):
    d = dispatch_durations(args.db)
    total = sum(sum(v) for v in d.values())
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))
    print("# rocprofv3 kernel trace summary (durations per dispatch)")
    for cmd in args.command:
        print(f"# command: {cmd}")
    print(f"# {'kernel':44s} {'calls':>8s} {'mean_us':>10s} {'min_us':>10s} {'max_us':>10s} "
          f"{'total_ms':>10s} {'pct':>6s}")
    for k, v in rows[: args.top]:
        print(f"  {k[:44]:44s} {len(v):8d} {sum(v) / len(v) / 1e3:10.3f} {min(v) / 1e3:10.3f} "
              f"{max(v) / 1e3:10.3f} {sum(v) / 1e6:10.3f} {100 * sum(v) / total:6.2f}")
    if args.bench_json:
        for line in open(args.bench_json):
            if line.startswith("{"):
                print(f"# bench line: {line.strip()}")


def counters(db: str, counter: str):
    c = sqlite3.connect(db)
    tabs = _tables(c)
    if "counters_collection" not in tabs:
        raise SystemExit(f"{db}: no counters_collection table among {tabs}")
    out = collections.defaultdict(list)
    q = "select kernel_name, counter_name, value from counters_collection"
    for n, cn, val in c.execute(q):
        if cn == counter:
            out[short_name(str(n))].append(float(val))
    return out


def pmc(args):
    from paper_1901_07374_amd.build import source_hash
    fetch = counters(args.fetch_db, "FETCH_SIZE")
    write = counters(args.write_db, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k or "copy_kernel" in k]
    if not copy:
        raise SystemExit("no device copy kernel among the counted dispatches")
    cf = max(max(fetch[k]) for k in copy)
    cw = max(max(write.get(k, [0.0])) for k in copy)
    f_fac = args.copy_bytes / (cf * 1024.0)
    w_fac = args.copy_bytes / (cw * 1024.0) if cw > 0 else float("nan")
    print("# rocprofv3 --pmc summary: HBM traffic per dispatch")
    for cmd in args.command:
        print(f"# command: {cmd}")
    print(f"# calibration: a device copy of {args.copy_bytes} bytes reads FETCH_SIZE = {cf:.0f} KiB"
          f" and writes WRITE_SIZE = {cw:.0f} KiB per dispatch")
    print(f"kernel_source_hash = {source_hash()}")
    print(f"fetch_scale = {f_fac:.4f}")
    print(f"write_scale = {w_fac:.4f}")
    for k in sorted(fetch):
        if not any(s in k for s in args.kernels):
            continue
        fv, wv = fetch[k], write.get(k, [])
        fm = sum(fv) / len(fv)
        wm = sum(wv) / len(wv) if wv else float("nan")
        hbm = (fm * f_fac + wm * w_fac) * 1024.0
        print(f"# {k}: dispatches {len(fv)}/{len(wv)}, FETCH_SIZE {fm:.1f} KiB, "
              f"WRITE_SIZE {wm:.1f} KiB")
        print(f"{k}_fetch_bytes_per_launch = {fm * f_fac * 1024.0:.0f}")
        print(f"{k}_write_bytes_per_launch = {wm * w_fac * 1024.0:.0f}")
        print(f"{k}_hbm_bytes_per_launch = {hbm:.0f}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--bench-json")
    t.add_argument("--top", type=int, default=16)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_db")
    p.add_argument("write_db")
    p.add_argument("--copy-bytes", type=int, required=True)
    p.add_argument("--command", action="append", default=[])
    p.add_argument("--kernels", nargs="*", default=["k_pass", "copyBuffer"])
    args = ap.parse_args(argv)
    trace(args) if args.mode == "trace" else pmc(args)


if __name__ == "__main__":
    sys.exit(main())
