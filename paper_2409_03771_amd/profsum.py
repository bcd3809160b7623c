"""Summaries of rocprofv3 output for the profiles folder.

    python -m paper_2409_03771_amd.profsum stats KERNEL_TRACE_CSV \\
        --cmd "<the rocprofv3 command>" --out profiles/NAME.md
    python -m paper_2409_03771_amd.profsum traffic \\
        --fetch FETCH_CSV --write WRITE_CSV \\
        --copy-fetch COPY_FETCH_CSV --copy-write COPY_WRITE_CSV \\
        --copy-bytes BYTES --cmd "<commands>" \\
        --out profiles/NAME.md --json profiles/NAME.json
    python -m paper_2409_03771_amd.profsum counters COUNTER_CSV \\
        --cmd "<the rocprofv3 command>" --out profiles/NAME.md

`stats` turns a --kernel-trace run (its per-dispatch trace) into a table of
the library's kernels, one row per kernel and grid size.  `traffic` turns
two --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) into HBM bytes per
launch, each scaled by what the same counter reads for a device copy of
known size, and records the hash of the kernel sources it was measured on:
the benchmark reports these bytes only while the sources are unchanged.
`counters` tabulates any other --pmc run.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/segment.hip", "csrc/cc.hip", "csrc/msc_internal.hpp")


def source_hash() -> str:
    """sha256 over the kernel sources, in a fixed order."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(rel.encode() + b"\0" + fh.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("msc::", "")
    n = re.sub(r"^void ", "", n)
    m = re.match(r"([A-Za-z_0-9]+)(<Cfg<([0-9, ]+)> >)?", n)
    if not m:
        return n[:60]
    base = m.group(1)
    if m.group(3):
        base += "<" + m.group(3).replace(" ", "") + ">"
    return base


def _ours(name: str) -> bool:
    return short_name(name).startswith("k_")


def _keyed(rows, name_col, grid_col):
    """(kernel, grid) -> rows; a kernel launched with several grid sizes
    (e.g. a pass and its rerun) is listed once per grid size."""
    by = collections.defaultdict(list)
    for r in rows:
        if _ours(r[name_col]):
            by[(short_name(r[name_col]), int(float(r[grid_col])))].append(r)
    grids = collections.Counter(k for k, _ in by)
    return {(f"{k} [grid {g}]" if grids[k] > 1 else k): v
            for (k, g), v in by.items()}


def cmd_stats(args):
    """Per-kernel durations from a --kernel-trace CSV (one row a dispatch)."""
    rows = list(csv.DictReader(open(args.csv)))
    by = _keyed(rows, "Kernel_Name", "Grid_Size_X")
    dur = {k: [(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
               for r in v] for k, v in by.items()}
    total = sum(sum(d) for d in dur.values())
    lines = [f"# Kernel trace: {args.title}", "", "Command:", "",
             "```", args.cmd, "```", "",
             "| kernel | calls | avg ms | min ms | max ms | share of library time |",
             "|---|---:|---:|---:|---:|---:|"]
    ranked = sorted(dur.items(), key=lambda kv: -sum(kv[1]))
    shown = ranked[:args.top] if args.top else ranked
    for k, d in shown:
        lines.append(
            f"| {k} | {len(d)} | {sum(d) / len(d) / 1e6:.3f} | "
            f"{min(d) / 1e6:.3f} | {max(d) / 1e6:.3f} | "
            f"{100 * sum(d) / total:.1f}% |")
    if len(shown) < len(ranked):
        rest = ranked[len(shown):]
        lines.append(f"| ({len(rest)} more rows) | "
                     f"{sum(len(d) for _, d in rest)} | | | | "
                     f"{100 * sum(sum(d) for _, d in rest) / total:.1f}% |")
    lines += ["", f"Sum over all launches of the library's kernels in the traced "
              f"run: {total / 1e6:.3f} ms.", "",
              f"Kernel sources sha256: `{source_hash()}`"]
    _write(args.out, lines)


def _per_kernel(path, counter):
    rows = [r for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter]
    acc = {k: [float(r["Counter_Value"]) for r in v]
           for k, v in _keyed(rows, "Kernel_Name", "Grid_Size").items()}
    # The copy kernel of the calibration run is not one of the library's.
    for r in rows:
        if not _ours(r["Kernel_Name"]):
            acc.setdefault(short_name(r["Kernel_Name"]), []).append(
                float(r["Counter_Value"]))
    return acc


def cmd_traffic(args):
    f = _per_kernel(args.fetch, "FETCH_SIZE")
    w = _per_kernel(args.write, "WRITE_SIZE")
    cf = _per_kernel(args.copy_fetch, "FETCH_SIZE")
    cw = _per_kernel(args.copy_write, "WRITE_SIZE")
    # The copy kernel: the dispatches that moved the most bytes.
    copy_f = max(sum(v) / len(v) for v in cf.values())
    copy_w = max(sum(v) / len(v) for v in cw.values())
    kib = args.copy_bytes / 1024.0
    ff, fw = kib / copy_f, kib / copy_w
    kernels = {}
    for k in sorted(set(f) | set(w)):
        if not k.startswith("k_"):
            continue
        fk = sum(f.get(k, [0])) / max(1, len(f.get(k, [])))
        wk = sum(w.get(k, [0])) / max(1, len(w.get(k, [])))
        kernels[k] = {"fetch_kib": fk, "write_kib": wk,
                      "hbm_bytes": (fk * ff + wk * fw) * 1024.0}
    rec = {"workload": args.title, "source_sha256": source_hash(),
           "copy_bytes": args.copy_bytes, "fetch_factor": ff,
           "write_factor": fw, "kernels": kernels}
    with open(args.json, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
        fh.write("\n")
    lines = [f"# HBM traffic: {args.title}", "", "Commands:", "", "```",
             args.cmd, "```", "",
             f"Calibration: a device copy of {args.copy_bytes} bytes reads "
             f"FETCH_SIZE = {copy_f:.0f} KiB and WRITE_SIZE = {copy_w:.0f} KiB "
             f"per dispatch, so FETCH_SIZE is scaled by {ff:.3f} and "
             f"WRITE_SIZE by {fw:.3f}.", "",
             "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch "
             "(scaled) |", "|---|---:|---:|---:|"]
    for k, v in kernels.items():
        lines.append(f"| {k} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | "
                     f"{v['hbm_bytes'] / 1e9:.3f} GB |")
    lines += ["", f"Kernel sources sha256: `{rec['source_sha256']}`"]
    _write(args.out, lines)


def cmd_counters(args):
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    rows = list(csv.DictReader(open(args.csv)))
    for k, v in _keyed(rows, "Kernel_Name", "Grid_Size").items():
        for r in v:
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for d in acc.values() for c in d})
    lines = [f"# Counters: {args.title}", "", "Command:", "", "```", args.cmd,
             "```", "", "Mean per dispatch.", "",
             "| kernel | " + " | ".join(names) + " |",
             "|---|" + "---:|" * len(names)]
    for k, d in acc.items():
        vals = [sum(d[c]) / len(d[c]) if d.get(c) else float("nan")
                for c in names]
        lines.append(f"| {k} | " + " | ".join(f"{v:.4g}" for v in vals) + " |")
    _write(args.out, lines)


def _write(path, lines):
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=0,
                   help="only the N rows with the most time")
    for p in (a,):
        p.add_argument("--cmd", required=True)
        p.add_argument("--out", required=True)
        p.add_argument("--title", default="")
    b = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--cmd",
              "--out", "--json"):
        b.add_argument(k, required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--title", default="")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--cmd", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--title", default="")
    args = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic,
     "counters": cmd_counters}[args.what](args)


if __name__ == "__main__":
    main()
