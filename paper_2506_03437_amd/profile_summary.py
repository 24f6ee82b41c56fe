"""Summaries of rocprofv3 result databases (rocpd SQLite) for profiles/.

    python -m paper_2506_03437_amd.profile_summary trace RUN_results.db
        per-kernel table: calls, average and total duration, share of GPU time
    python -m paper_2506_03437_amd.profile_summary pmc --kernel NAME \\
            --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db --copy-bytes B
        HBM bytes per dispatch of kernel NAME from FETCH_SIZE and WRITE_SIZE
        (KiB per dispatch), each scaled by what the same counter reads for a
        plain copy of B bytes (the largest copy dispatch in the copy runs)

Reads the databases with sqlite3 only; prints markdown.
"""

from __future__ import annotations

import argparse
import collections
import sqlite3
import sys


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def kernel_table(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = collections.defaultdict(lambda: [0, 0.0])
    for n, d in rows:
        a = agg[_short(n)]
        a[0] += 1
        a[1] += d
    total = sum(v[1] for v in agg.values())
    out = []
    for n, (calls, dur) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append((n, calls, dur / calls / 1e3, dur / 1e6, 100.0 * dur / total))
    return out


def counter_per_dispatch(db: str, kernel: str, counter: str) -> tuple:
    """(mean counter value per dispatch of kernels whose name contains `kernel`, dispatches)."""
    c = sqlite3.connect(db)
    per = collections.defaultdict(float)
    for n, cn, v, did in c.execute("select name, counter_name, counter_value, dispatch_id from pmc_events"):
        if cn == counter and kernel in n:
            per[did] += v
    if not per:
        return 0.0, 0
    return sum(per.values()) / len(per), len(per)


def copy_counter(db: str, counter: str) -> float:
    """Counter value (KiB) of the largest copy dispatch of a calibration run."""
    c = sqlite3.connect(db)
    per = collections.defaultdict(float)
    for n, cn, v, did in c.execute("select name, counter_name, counter_value, dispatch_id from pmc_events"):
        if cn == counter and "copy" in n.lower():
            per[did] += v
    return max(per.values()) if per else 0.0


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=15)
    p = sub.add_parser("pmc")
    p.add_argument("--kernel", required=True)
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--copy-fetch", required=True)
    p.add_argument("--copy-write", required=True)
    p.add_argument("--copy-bytes", type=float, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print("| kernel | calls | average (us) | total (ms) | share of GPU time |")
        print("|---|---|---|---|---|")
        for n, calls, avg, tot, pct in kernel_table(a.db)[: a.top]:
            print(f"| `{n}` | {calls} | {avg:.1f} | {tot:.2f} | {pct:.2f}% |")
        return 0
    kib = a.copy_bytes / 1024.0
    cf = copy_counter(a.copy_fetch, "FETCH_SIZE")
    cw = copy_counter(a.copy_write, "WRITE_SIZE")
    ff = kib / cf if cf else float("nan")
    fw = kib / cw if cw else float("nan")
    f, nf = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    w, nw = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    fetch_b = f * ff * 1024.0
    write_b = w * fw * 1024.0
    print(f"copy calibration: {a.copy_bytes:.0f}-byte copy reads FETCH_SIZE {cf:.1f} KiB (factor {ff:.4f}), "
          f"WRITE_SIZE {cw:.1f} KiB (factor {fw:.4f})")
    print(f"{a.kernel}: FETCH_SIZE {f:.1f} KiB per dispatch ({nf} dispatches) -> {fetch_b / 1e9:.4f} GB")
    print(f"{a.kernel}: WRITE_SIZE {w:.1f} KiB per dispatch ({nw} dispatches) -> {write_b / 1e9:.4f} GB")
    print(f"traffic_bytes_per_launch = {fetch_b + write_b:.0f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
