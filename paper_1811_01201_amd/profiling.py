"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1811_01201_amd.profiling stats  KERNEL_STATS_CSV
    python -m paper_1811_01201_amd.profiling counters COUNTER_CSV [...]
    python -m paper_1811_01201_amd.profiling traffic --fetch CSV --write CSV \\
        --kernel REGEX --copy-bytes N [--out FILE]

``traffic`` turns two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE; KiB per
dispatch) into HBM bytes per launch of the kernels matching REGEX.  Each
counter is scaled by what it reads for the copy kernel of the same run,
whose bytes are known (``--copy-bytes`` read and as many written): the
ratio known/measured corrects for what the counter does not see.  The
summary records the SHA-256 of the sources that define the phase kernels;
``bench.py`` reports the traffic only while they are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/apsp_internal.h", "csrc/apsp_single.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without its parameter list (template arguments kept)."""
    name = name.strip()
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(name[i], 0)
            if depth == 0:
                name = name[:i]
                break
    return name.replace("void ", "").replace("apsp::", "").strip()


def kernel_stats(path: str):
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                     "avg_ms": float(r["AverageNs"]) / 1e6, "total_ms": float(r["TotalDurationNs"]) / 1e6,
                     "percent": float(r["Percentage"])})
    return rows


def counters(paths):
    """{kernel: {"dispatches": d, "avg_ms": t, counter: per-dispatch value}}"""
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(dict)
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            key = (path, r["Dispatch_Id"])
            vals[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k][key] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = {}
    for k, v in vals.items():
        nd = len(disp[k])
        npaths = len({p for p, _ in disp[k]})
        per_pass = nd / npaths
        row = {"dispatches": per_pass, "avg_ms": sum(disp[k].values()) / nd / 1e6}
        for c, x in v.items():
            row[c] = x / per_pass
        out[k] = row
    return out


def largest_dispatch(path, kernel_pred, counter):
    """(kernel, value) of the dispatch with the largest `counter` among the
    kernels kernel_pred accepts."""
    best = (None, -1.0)
    per = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        if r["Counter_Name"] != counter or not kernel_pred(k):
            continue
        per[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = k
    for d, v in per.items():
        if v > best[1]:
            best = (names[d], v)
    return best


def traffic(fetch_csv, write_csv, kernel_regex, copy_bytes):
    """Per-launch HBM bytes of the kernels matching kernel_regex.  The scale
    comes from the largest copy dispatch of each run (the input restore of
    copy_bytes); smaller copies of the same kernel (scalars read back) are
    ignored."""
    f = counters([fetch_csv])
    w = counters([write_csv])
    is_copy = lambda k: "copyBuffer" in k
    ck, fetch_kib = largest_dispatch(fetch_csv, is_copy, "FETCH_SIZE")
    _, write_kib = largest_dispatch(write_csv, is_copy, "WRITE_SIZE")
    if ck is None or fetch_kib <= 0 or write_kib <= 0:
        raise SystemExit("no copy kernel in the counter run")
    f_scale = copy_bytes / (fetch_kib * 1024.0)
    w_scale = copy_bytes / (write_kib * 1024.0)
    rx = re.compile(kernel_regex)
    ks = [k for k in f if rx.search(k)]
    res = {}
    for k in ks:
        fb = f[k]["FETCH_SIZE"] * 1024.0 * f_scale
        wb = w[k]["WRITE_SIZE"] * 1024.0 * w_scale
        res[k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb, "dispatches": f[k]["dispatches"],
                  "avg_ms": f[k]["avg_ms"]}
    return {"fetch_scale": f_scale, "write_scale": w_scale, "copy_kernel": ck, "kernels": res}


def read_traffic_file(path):
    """key=value lines of a traffic summary -> dict (None if absent)."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--command", default="")
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        for r in kernel_stats(a.csv):
            print(f"{r['name'][:80]:80s} calls={r['calls']:5d} avg_ms={r['avg_ms']:.4f} share={r['percent']:.2f}%")
    elif a.cmd == "counters":
        for k, row in counters(a.csv).items():
            print(k)
            for name, v in sorted(row.items()):
                print(f"    {name:28s} {v:.6g}")
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.copy_bytes)
        if a.out and len(res["kernels"]) != 1:
            raise SystemExit(f"--kernel must select one kernel for --out, got {sorted(res['kernels'])}")
        lines = [f"# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE",
                 f"# command: {a.command}" if a.command else "# command: (not recorded)",
                 f"copy_kernel={res['copy_kernel']}", f"copy_bytes={a.copy_bytes:.0f}",
                 f"fetch_scale={res['fetch_scale']:.4f}", f"write_scale={res['write_scale']:.4f}",
                 f"source_sha256={kernel_source_hash()}"]
        for k, r in res["kernels"].items():
            lines.append(f"# kernel {k}: dispatches={r['dispatches']:.0f} avg_ms={r['avg_ms']:.4f}")
            lines.append(f"kernel={k}")
            lines.append(f"fetch_bytes_per_launch={r['fetch_bytes']:.0f}")
            lines.append(f"write_bytes_per_launch={r['write_bytes']:.0f}")
            lines.append(f"traffic_bytes_per_launch={r['bytes']:.0f}")
        text = "\n".join(lines) + "\n"
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)


if __name__ == "__main__":
    main()
