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
  sq:    python -m paper_1901_07374_amd.rocprof_summary sq A.db [B.db ...]
         SQ counters (instruction counts, busy and wait cycles, LDS bank
         conflicts) per kernel with derived shares.
  --last N keeps each kernel's last N dispatches (the timed steps of a run
  whose untimed steps use the same kernels).
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
            # rows are read as stored (views over large tables sort slowly)
            # and put in dispatch order here
            rows = []
            for k, (n, b, e) in enumerate(c.execute(f'select "{name}", "{beg}", "{end}" from "{t}"')):
                rows.append((float(b), str(n), float(e) - float(b)))
                if k % 200000 == 0:
                    print(f"# read {k} dispatches of {db}", file=sys.stderr, flush=True)
            rows.sort()
            out = collections.defaultdict(list)
            names = {}
            for _, n, d in rows:
                if n not in names:
                    names[n] = short_name(n)
                out[names[n]].append(d)
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


def last(d, k):
    """Each kernel's last k dispatches (k <= 0: all)."""
    return {n: (v[-k:] if k > 0 else v) for n, v in d.items()}


def trace(args):
    d = last(dispatch_durations(args.db), args.last)
    total = sum(sum(v) for v in d.values())
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))
    print("# rocprofv3 kernel trace summary (durations per dispatch)"
          + (f"; each kernel's last {args.last} dispatches" if args.last > 0 else ""))
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
    return counter_table(db, [counter])[counter]


_TABLE_CACHE = {}


def counter_table(db: str, names):
    """{counter: {kernel: [value per dispatch, in dispatch order]}}, from one
    pass over the counter view (rows read as stored, ordered here by the
    dispatch id when the view has one)."""
    if db not in _TABLE_CACHE:
        c = sqlite3.connect(db)
        cols = _cols(c, "counters_collection")
        key = next((k for k in ("dispatch_id", "correlation_id", "start", "start_ns")
                    if k in cols), None)
        sel = f'"{key}", ' if key else ""
        rows = []
        q = f"select {sel}kernel_name, counter_name, value from counters_collection"
        for k, r in enumerate(c.execute(q)):
            rows.append((float(r[0]) if key else k, str(r[-3]), str(r[-2]), float(r[-1])))
            if k % 200000 == 0:
                print(f"# read {k} counter rows of {db}", file=sys.stderr, flush=True)
        rows.sort(key=lambda x: x[0])
        tab = collections.defaultdict(lambda: collections.defaultdict(list))
        short = {}
        for _, n, cn, v in rows:
            if n not in short:
                short[n] = short_name(n)
            tab[cn][short[n]].append(v)
        _TABLE_CACHE[db] = tab
    tab = _TABLE_CACHE[db]
    return {cn: tab.get(cn, {}) for cn in names}


def pmc(args):
    from paper_1901_07374_amd.build import source_hash
    fetch = last(counters(args.fetch_db, "FETCH_SIZE"), args.last)
    write = last(counters(args.write_db, "WRITE_SIZE"), args.last)
    copy = [k for k in fetch if "copyBuffer" in k or "copy_kernel" in k]
    if not copy:
        raise SystemExit("no device copy kernel among the counted dispatches")
    # the calibration copy is the run's last copy (other copies, e.g. the
    # autotuner's state saves, have other sizes)
    cf = fetch[copy[0]][-1]
    cw = write.get(copy[0], [0.0])[-1]
    f_fac = args.copy_bytes / (cf * 1024.0)
    w_fac = args.copy_bytes / (cw * 1024.0) if cw > 0 else float("nan")
    print("# rocprofv3 --pmc summary: HBM traffic per dispatch")
    for cmd in args.command:
        print(f"# command: {cmd}")
    print(f"# calibration: a device copy of {args.copy_bytes} bytes reads FETCH_SIZE = {cf:.0f} KiB"
          f" and writes WRITE_SIZE = {cw:.0f} KiB per dispatch")
    if args.last > 0:
        print(f"# per kernel: its last {args.last} dispatches (the timed steps)")
    print(f"kernel_source_hash = {source_hash()}")
    print(f"fetch_scale = {f_fac:.4f}")
    print(f"write_scale = {w_fac:.4f}")
    print("# kernels counted: " + "; ".join(sorted(k[:48] for k in fetch)))
    gat = [k for k in fetch if "gather" in k.lower() or "index" in k.lower()]
    if gat and args.gather_read_bytes:
        gf = max(max(fetch[k]) for k in gat)
        print(f"# gather calibration: {gat[0][:60]} reads {args.gather_read_bytes} bytes "
              f"(64-byte rows in random order, each once, plus 8-byte indices) and FETCH_SIZE "
              f"says {gf:.0f} KiB")
        print(f"fetch_scale_gather = {args.gather_read_bytes / (gf * 1024.0):.4f}")
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


def sq(args):
    """SQ counters per kernel (sum over the kept dispatches), with the
    derived rates: VALU busy = SQ_ACTIVE_INST_VALU / (SQ_BUSY_CU_CYCLES or
    SQ_WAVE_CYCLES share), waits, LDS bank conflicts per LDS instruction."""
    from paper_1901_07374_amd.build import source_hash
    tab = {}
    for db in args.dbs:
        counter_table(db, [])
        names = sorted(_TABLE_CACHE[db])
        for cn, per in counter_table(db, names).items():
            for k, v in last(per, args.last).items():
                tab.setdefault(k, {})[cn] = (sum(v), len(v))
    print("# rocprofv3 --pmc summary: SQ counters per kernel, summed over dispatches")
    for cmd in args.command:
        print(f"# command: {cmd}")
    if args.last > 0:
        print(f"# per kernel: its last {args.last} dispatches (the timed steps)")
    print(f"kernel_source_hash = {source_hash()}")
    for k in sorted(tab):
        if not any(s in k for s in args.kernels):
            continue
        row = tab[k]
        print(f"# {k}")
        for cn in sorted(row):
            tot, cnt = row[cn]
            print(f"{k}_{cn} = {tot / cnt:.6g}   # mean per dispatch over {cnt}")
        g = {cn: row[cn][0] / row[cn][1] for cn in row}
        if "SQ_INSTS_VALU" in g and "SQ_WAVES" in g and g["SQ_WAVES"] > 0:
            print(f"{k}_valu_insts_per_wave = {g['SQ_INSTS_VALU'] / g['SQ_WAVES']:.1f}")
        if "SQ_ACTIVE_INST_VALU" in g and "SQ_WAVE_CYCLES" in g and g["SQ_WAVE_CYCLES"] > 0:
            print(f"{k}_valu_active_share_of_wave_cycles = "
                  f"{g['SQ_ACTIVE_INST_VALU'] / g['SQ_WAVE_CYCLES']:.4f}")
        if "SQ_WAIT_INST_ANY" in g and "SQ_WAVE_CYCLES" in g and g["SQ_WAVE_CYCLES"] > 0:
            print(f"{k}_wait_share_of_wave_cycles = "
                  f"{g['SQ_WAIT_INST_ANY'] / g['SQ_WAVE_CYCLES']:.4f}")
        if "SQ_LDS_BANK_CONFLICT" in g and "SQ_INSTS_LDS" in g and g["SQ_INSTS_LDS"] > 0:
            print(f"{k}_lds_bank_conflict_cycles_per_lds_inst = "
                  f"{g['SQ_LDS_BANK_CONFLICT'] / g['SQ_INSTS_LDS']:.3f}")


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
    p.add_argument("--kernels", nargs="*", default=["k_pass", "copyBuffer", "index"])
    p.add_argument("--gather-read-bytes", type=int, default=0)
    p.add_argument("--last", type=int, default=0)
    t.add_argument("--last", type=int, default=0,
                   help="summarise each kernel's last N dispatches only (0: all)")
    q = sub.add_parser("sq")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--command", action="append", default=[])
    q.add_argument("--kernels", nargs="*", default=["k_pass"])
    q.add_argument("--last", type=int, default=0)
    args = ap.parse_args(argv)
    {"trace": trace, "pmc": pmc, "sq": sq}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
