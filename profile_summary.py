"""Summaries of rocprofv3 results databases (kernel durations, PMC counters).

    python profile_summary.py trace DB [--split-gap-ms G]
    python profile_summary.py window DB --kernel NAME --last N [--prefix]
    python profile_summary.py pmc FETCH_DB WRITE_DB --kernel NAME [--copy-bytes B] [--prefix --last N]

The window mode summarises the dispatches from the first of the last N
dispatches of the named kernel to the end of the trace (bench.py reports how
many launches of its dominant kernel fall in its timed steps), and that
kernel's average duration over those N dispatches.

The pmc mode reports FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the named
kernel, scaled by the ratio of the known byte count of a plain device copy
to what the same counters read for that copy kernel; with --prefix every
kernel whose name starts with NAME counts as one, and --last N averages over
its last N dispatches only (the timed steps).
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics


def segments(db, gap_ms):
    """Dispatches (name, duration) split where the device sat idle for more
    than gap_ms between two kernels (e.g. between two runs of one program)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, duration from kernels order by start").fetchall()
    segs, cur, last = [], [], None
    for name, start, end, dur in rows:
        if last is not None and (start - last) / 1e6 > gap_ms and cur:
            segs.append(cur)
            cur = []
        cur.append((name, dur))
        last = end if last is None else max(last, end)
    if cur:
        segs.append(cur)
    return segs


def trace(db, top=20, rows=None):
    if rows is None:
        con = sqlite3.connect(db)
        rows = con.execute("select name, duration from kernels").fetchall()
    agg = {}
    for name, dur in rows:
        agg.setdefault(name.split("(")[0], []).append(dur)
    tot = sum(sum(v) for v in agg.values())
    out = []
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append((name, len(v), sum(v) / 1e6, statistics.mean(v) / 1e6, 100.0 * sum(v) / tot))
    return out, tot / 1e6


def window(db, kernel, last, prefix=False):
    """Dispatches from the first of the last `last` dispatches of `kernel`
    (its name, or with prefix=True every name that starts with it, e.g. all
    tile shapes of a template) onwards, and those dispatches' mean duration (ms)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, duration from kernels order by start").fetchall()
    match = (lambda nm: nm.startswith(kernel)) if prefix else (lambda nm: nm == kernel)
    hits = [i for i, (name, _, _) in enumerate(rows) if match(name.split("(")[0])]
    if len(hits) < last:
        raise SystemExit(f"{kernel}: {len(hits)} dispatches in the trace, fewer than {last}")
    first = hits[-last]
    sel = [(name, dur) for name, _, dur in rows[first:]]
    mean = statistics.mean(rows[i][2] for i in hits[-last:]) / 1e6
    return sel, mean


def pmc(db, counter, group=None, last=0):
    """{kernel: [counter value per dispatch]} (summed over counter instances).
    group: every kernel name starting with it counts as that one name (e.g.
    all tile shapes of a template); last > 0 keeps only the last `last`
    dispatches (in dispatch order) of each name."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select k.name, p.dispatch_id, p.counter_value from pmc_events p join kernels k on p.dispatch_id = k.dispatch_id "
        "where p.counter_name = ?", (counter,)).fetchall()
    agg = {}
    for name, did, val in rows:
        key = name.split("(")[0]
        if group and key.startswith(group):
            key = group
        agg.setdefault(key, {}).setdefault(did, 0.0)
        agg[key][did] += float(val)
    out = {}
    for k, v in agg.items():
        vals = [v[d] for d in sorted(v)]
        out[k] = vals[-last:] if last > 0 and k == group else vals
    return out


def last_dispatch(db, counter, substr):
    """(name, counter value in bytes) of the last dispatch whose kernel name
    contains substr (not one of this library's kernels)."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select k.name, p.dispatch_id, p.counter_value from pmc_events p join kernels k on p.dispatch_id = k.dispatch_id "
        "where p.counter_name = ? order by p.dispatch_id", (counter,)).fetchall()
    per = {}
    for name, did, val in rows:
        if substr.lower() in name.lower() and "eahp" not in name:
            per.setdefault(did, [name.split("(")[0], 0.0])[1] += float(val)
    if not per:
        return None, float("nan")
    name, val = per[max(per)]
    return name, val * 1024.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "window", "pmc"])
    ap.add_argument("dbs", nargs="+")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--copy-bytes", type=float, default=536870912.0)
    ap.add_argument("--copy-kernel", default="copy")
    ap.add_argument("--split-gap-ms", type=float, default=0.0,
                    help="report separately the stretches of dispatches separated by idle gaps above this")
    ap.add_argument("--min-dispatches", type=int, default=100)
    ap.add_argument("--last", type=int, default=0)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--prefix", action="store_true", help="window: match every kernel name starting with --kernel")
    a = ap.parse_args()
    if a.mode == "window":
        sel, mean = window(a.dbs[0], a.kernel, a.last, a.prefix)
        rows, tot = trace(a.dbs[0], top=a.top, rows=sel)
        print(f"window: {len(sel)} dispatches from the first of the last {a.last} dispatches of {a.kernel}")
        print(f"{a.kernel}: mean duration over those {a.last} dispatches {mean:.4f} ms")
        print(f"total kernel time {tot:.3f} ms")
        print("| kernel | calls | total ms | avg ms | % |")
        print("|---|---|---|---|---|")
        for name, n, t, avg, pct in rows:
            print(f"| {name} | {n} | {t:.3f} | {avg:.4f} | {pct:.1f} |")
        return
    if a.mode == "trace":
        segs = segments(a.dbs[0], a.split_gap_ms) if a.split_gap_ms > 0 else [None]
        if a.split_gap_ms > 0:
            segs = [sg for sg in segs if len(sg) >= a.min_dispatches]
        for i, sg in enumerate(segs):
            rows, tot = trace(a.dbs[0], rows=sg)
            if sg is not None:
                print(f"\nsegment {i + 1} of {len(segs)}: {len(sg)} dispatches")
            print(f"total kernel time {tot:.3f} ms")
            print("| kernel | calls | total ms | avg ms | % |")
            print("|---|---|---|---|---|")
            for name, n, t, avg, pct in rows:
                print(f"| {name} | {n} | {t:.3f} | {avg:.4f} | {pct:.1f} |")
        return
    group = a.kernel if a.prefix else None
    fetch = pmc(a.dbs[0], "FETCH_SIZE", group, a.last)
    write = pmc(a.dbs[1], "WRITE_SIZE", group, a.last)
    # the copy probe is the last dispatch of a copy kernel (bench.py --copy-probe
    # issues it after everything else)
    ck, cf = last_dispatch(a.dbs[0], "FETCH_SIZE", a.copy_kernel)
    _, cw = last_dispatch(a.dbs[1], "WRITE_SIZE", a.copy_kernel)
    sf, sw = a.copy_bytes / cf, a.copy_bytes / cw
    print(f"copy probe ({ck}): FETCH {cf:.6g} B, WRITE {cw:.6g} B for a {a.copy_bytes:.6g} B copy "
          f"-> scale FETCH x{sf:.4f}, WRITE x{sw:.4f}")
    print("| kernel | dispatches | FETCH MB/dispatch (scaled) | WRITE MB/dispatch (scaled) | total MB |")
    print("|---|---|---|---|---|")
    for k in sorted(fetch, key=lambda x: -statistics.mean(fetch[x])):
        if a.kernel and a.kernel not in k:
            continue
        f = statistics.mean(fetch[k]) * 1024.0 * sf
        w = statistics.mean(write.get(k, [0.0])) * 1024.0 * sw
        print(f"| {k} | {len(fetch[k])} | {f / 1e6:.3f} | {w / 1e6:.3f} | {(f + w) / 1e6:.3f} |")


if __name__ == "__main__":
    main()
