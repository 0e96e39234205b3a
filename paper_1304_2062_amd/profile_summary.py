"""Summaries of rocprofv3 output for the committed performance records.

Two inputs, both CSV directories written by rocprofv3 (``-f csv``):

* a ``--kernel-trace --stats`` run  -> per-kernel call count and average
  duration (``*_kernel_stats.csv``);
* two ``--pmc`` runs, one with ``FETCH_SIZE`` and one with ``WRITE_SIZE``
  (``*_counter_collection.csv``), of a workload that also performs one plain
  device-to-device copy of known size (``__amd_rocclr_copyBuffer``).  The
  counters read that copy's bytes with some scale (the request-size
  accounting of the counter); the ratio known / counted is applied to every
  kernel, giving HBM-side bytes per dispatch.

Usage:
    python -m paper_1304_2062_amd.profile_summary stats <dir> --cmd "<command>" > profiles/x.md
    python -m paper_1304_2062_amd.profile_summary traffic <fetch_dir> <write_dir> --copy-bytes B \\
        --cmd "<commands>" [--json out.json] > profiles/y.md
    python -m paper_1304_2062_amd.profile_summary sq <dir> [<dir> ...] --cmd "<commands>" > profiles/z.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(name: str) -> str:
    """Kernel name without the argument list and namespace."""
    base = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("se2n::", "")
    return re.sub(r"\s+", "", base)


def kernel_source_hash() -> str:
    """Hash of the sources the single-image path is built from (kernels, tile
    bodies, FFT core, host runtime); a traffic record is valid only for these.
    The batched and corrector sources do not enter it."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if os.path.basename(p).startswith(("se2n_batch", "se2n_cnn")):
            continue
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(dirname: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    return sorted(hits)[0]


def stats(dirname: str) -> list[dict]:
    rows = list(csv.DictReader(open(_find(dirname, "kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append({
            "kernel": short_name(r["Name"]),
            "calls": int(r["Calls"]),
            "avg_us": float(r["AverageNs"]) / 1e3,
            "total_ms": float(r["TotalDurationNs"]) / 1e6,
            "pct": float(r["Percentage"]),
        })
    return out


def counters(dirname: str) -> dict[str, list[float]]:
    rows = list(csv.DictReader(open(_find(dirname, "counter_collection.csv"))))
    agg: dict[str, list[float]] = defaultdict(list)
    for r in rows:
        agg[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return agg


def named_counters(dirname: str) -> dict[str, dict[str, list[float]]]:
    """{kernel: {counter: [value per dispatch]}} of a --pmc run with several counters."""
    rows = list(csv.DictReader(open(_find(dirname, "counter_collection.csv"))))
    agg: dict[str, dict[str, list[float]]] = defaultdict(lambda: defaultdict(list))
    for r in rows:
        agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--cmd", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--cmd", required=True)
    b.add_argument("--json")
    c = sub.add_parser("sq", help="per-kernel averages of SQ counters from one or more --pmc runs")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--cmd", required=True)
    c.add_argument("--kernels", default="", help="comma-separated kernel name prefixes to keep")
    args = ap.parse_args(argv)

    if args.mode == "sq":
        keep = [k for k in args.kernels.split(",") if k]
        table: dict[str, dict[str, float]] = defaultdict(dict)
        names: list[str] = []
        for d in args.dirs:
            for k, cs in named_counters(d).items():
                if keep and not any(k.startswith(p) for p in keep):
                    continue
                for cn, vals in cs.items():
                    table[k][cn] = sum(vals) / len(vals)
                    if cn not in names:
                        names.append(cn)
        print("# SQ counters per dispatch (rocprofv3 --pmc)\n")
        print(f"Commands:\n\n    {args.cmd}\n")
        print(f"Source hash of the single-image kernels: {kernel_source_hash()}\n")
        print("| kernel | " + " | ".join(names) + " |")
        print("|---|" + "---|" * len(names))
        for k in sorted(table):
            print(f"| `{k}` | " + " | ".join(f"{table[k].get(n, float('nan')):.4g}" for n in names) + " |")
        return 0

    if args.mode == "stats":
        st = stats(args.dir)
        print("# rocprofv3 kernel trace summary\n")
        print(f"Command:\n\n    {args.cmd}\n")
        print("| kernel | calls | average (us) | total (ms) | % |")
        print("|---|---|---|---|---|")
        for r in st:
            print(f"| `{r['kernel']}` | {r['calls']} | {r['avg_us']:.2f} | {r['total_ms']:.3f} | {r['pct']:.2f} |")
        return 0

    fetch = counters(args.fetch_dir)
    write = counters(args.write_dir)
    copy = "__amd_rocclr_copyBuffer"
    # the largest copy dispatch is the calibration copy
    f_copy = max(fetch[copy]) * 1024.0
    w_copy = max(write[copy]) * 1024.0
    f_scale = args.copy_bytes / f_copy
    w_scale = args.copy_bytes / w_copy
    rec = {"copy_bytes": args.copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
           "source_hash": kernel_source_hash(), "kernels": {}}
    print("# HBM traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n")
    print(f"Commands:\n\n    {args.cmd}\n")
    print(f"Calibration: one device-to-device copy of {args.copy_bytes} bytes reads "
          f"FETCH_SIZE = {f_copy / 1024:.0f} KiB and WRITE_SIZE = {w_copy / 1024:.0f} KiB; "
          f"scale factors {f_scale:.3f} (fetch) and {w_scale:.3f} (write) convert the counters "
          f"to bytes.\n")
    print("| kernel | dispatches | fetch (MB) | write (MB) | fetch+write (MB) |")
    print("|---|---|---|---|---|")
    for k in fetch:
        if k == copy:
            continue
        fv = fetch[k]
        wv = write.get(k, [0.0])
        fb = sum(fv) / len(fv) * 1024.0 * f_scale
        wb = sum(wv) / len(wv) * 1024.0 * w_scale
        rec["kernels"][k] = {"fetch_bytes": fb, "write_bytes": wb, "dispatches": len(fv)}
        print(f"| `{k}` | {len(fv)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rec, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
