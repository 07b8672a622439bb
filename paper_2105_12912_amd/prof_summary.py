"""Summaries of rocprofv3 output for the kernels of this library.

Two inputs are understood:

* a ``--kernel-trace --stats`` directory (``*_kernel_stats.csv``): per-kernel
  call count and average / min / max duration;
* ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` directories
  (``*_counter_collection.csv``, one pass per counter), together with the same
  two passes over a plain device copy of known size.  The copy gives the scale
  from counter units (KiB) to bytes: ``factor = copy_bytes / counter_bytes``.
  Per-kernel HBM bytes per dispatch are then ``(FETCH + WRITE) * factor``.

A third form averages any other counters per dispatch (``--pmc`` passes of
up to eight SQ counters each), for a list of kernels.

Usage::

  python -m paper_2105_12912_amd.prof_summary stats DIR
  python -m paper_2105_12912_amd.prof_summary traffic --fetch DIR --write DIR \\
      --copy-fetch DIR --copy-write DIR --copy-bytes N [--json OUT --key WORKLOAD]
  python -m paper_2105_12912_amd.prof_summary counters DIR [DIR ...] --kernels K1,K2,...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# source files whose text determines each kernel's memory traffic
KERNEL_SOURCES = {
    "k_construct": ["paper_2105_12912_amd/csrc/k_quant.hip"],
    "k_reconstruct": ["paper_2105_12912_amd/csrc/k_recon.hip"],
    "k_reconstruct3": ["paper_2105_12912_amd/csrc/k_recon.hip"],
    "k_huff_decode": ["paper_2105_12912_amd/csrc/k_huffman.hip"],
    "k_huff_write": ["paper_2105_12912_amd/csrc/k_huffman.hip"],
    "k_huff_bits": ["paper_2105_12912_amd/csrc/k_huffman.hip"],
    "k_range": ["paper_2105_12912_amd/csrc/k_quant.hip"],
    "k_rle_count": ["paper_2105_12912_amd/csrc/k_rle.hip"],
    "k_rle_write": ["paper_2105_12912_amd/csrc/k_rle.hip"],
    "k_rle_expand": ["paper_2105_12912_amd/csrc/k_rle.hip"],
}
COMMON_SOURCES = ["paper_2105_12912_amd/csrc/ebc_dev.h", "paper_2105_12912_amd/csrc/ebc_types.h"]


def source_hash(kernel: str) -> str | None:
    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for p in files + COMMON_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel base name without template arguments or parameter list."""
    n = name.strip()
    for sep in ("(", "<"):
        i = n.find(sep)
        if i > 0:
            n = n[:i]
    return n.split("::")[-1].strip()


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def kernel_stats(d: str):
    rows = []
    with open(_find(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append(dict(name=r["Name"], calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                             min_ns=float(r["MinNs"]), max_ns=float(r["MaxNs"]),
                             pct=float(r["Percentage"])))
    return rows


def counter_per_dispatch(d: str, counter: str):
    """{kernel short name: [value per dispatch]} for one counter pass."""
    out = defaultdict(list)
    per = defaultdict(float)
    names = {}
    with open(_find(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            key = r.get("Dispatch_Id") or r.get("Correlation_Id")
            per[key] += float(r["Counter_Value"])
            names[key] = short_name(r["Kernel_Name"])
    for k, v in per.items():
        out[names[k]].append(v)
    return out


def _avg(v):
    return sum(v) / len(v) if v else 0.0


def cmd_stats(a):
    rows = kernel_stats(a.dir)
    print(f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
    for r in rows:
        print(f"{short_name(r['name'])[:40]:40s} {r['calls']:6d} {r['avg_ns'] / 1e3:10.1f} "
              f"{r['min_ns'] / 1e3:10.1f} {r['max_ns'] / 1e3:10.1f} {r['pct']:6.2f}")


def cmd_traffic(a):
    fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(a.write, "WRITE_SIZE")
    cf = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw = counter_per_dispatch(a.copy_write, "WRITE_SIZE")
    # the copy kernel is the one with the largest per-dispatch fetch
    ck = max(cf, key=lambda k: _avg(cf[k]))
    f_fetch = a.copy_bytes / (_avg(cf[ck]) * 1024.0)
    f_write = a.copy_bytes / (_avg(cw.get(ck, [0.0])) * 1024.0) if cw.get(ck) else f_fetch
    print(f"copy kernel {ck}: {a.copy_bytes} B each way; FETCH_SIZE {_avg(cf[ck]):.0f} KiB, "
          f"WRITE_SIZE {_avg(cw.get(ck, [0])):.0f} KiB per dispatch -> factors fetch {f_fetch:.4f} "
          f"write {f_write:.4f}")
    print(f"{'kernel':28s} {'dispatches':>10s} {'fetch_MB':>10s} {'write_MB':>10s} {'hbm_MB':>10s}")
    rec = {}
    for k in sorted(fetch, key=lambda k: -_avg(fetch[k])):
        fb = _avg(fetch[k]) * 1024.0 * f_fetch
        wb = _avg(write.get(k, [0.0])) * 1024.0 * f_write
        print(f"{k[:28]:28s} {len(fetch[k]):10d} {fb / 1e6:10.2f} {wb / 1e6:10.2f} {(fb + wb) / 1e6:10.2f}")
        rec[k] = dict(fetch_bytes=round(fb), write_bytes=round(wb), bytes_per_launch=round(fb + wb),
                      source_hash=source_hash(k))
    if a.json:
        data = {}
        if os.path.exists(a.json):
            with open(a.json) as f:
                data = json.load(f)
        data[a.key] = dict(copy_factor_fetch=f_fetch, copy_factor_write=f_write, kernels=rec)
        with open(a.json, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


def counter_names(d: str):
    with open(_find(d, "counter_collection.csv")) as f:
        return sorted({r["Counter_Name"] for r in csv.DictReader(f)})


def cmd_counters(a):
    kernels = [k for k in a.kernels.split(",") if k]
    table = defaultdict(dict)
    for d in a.dirs:
        for c in counter_names(d):
            per = counter_per_dispatch(d, c)
            for k in kernels:
                if per.get(k):
                    table[k][c] = (_avg(per[k]), len(per[k]))
    for k in kernels:
        if not table[k]:
            continue
        print(k)
        for c, (v, n) in sorted(table[k].items()):
            print(f"  {c:28s} {v:18.0f}   ({n} dispatches)")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--json")
    t.add_argument("--key", default="nyx512")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernels", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
