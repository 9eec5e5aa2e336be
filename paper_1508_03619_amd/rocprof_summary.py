"""Summarise rocprofv3 output for the committed profiles.

Usage:
  python -m paper_1508_03619_amd.rocprof_summary stats <kernel_stats.csv> <out.txt> --cmd "<command>"
  python -m paper_1508_03619_amd.rocprof_summary traffic <fetch_counter_collection.csv>
         <write_counter_collection.csv> <out.json> --kernel k_bfs_persistent --copy-bytes N --cmd "..."
  python -m paper_1508_03619_amd.rocprof_summary counters <counter_collection.csv>... --out <out.txt>
         --kernel k_bfs_persistent --kernel k_msbfs --cmd "..."

The traffic summary scales the counters of the search kernel by the ratio
(known bytes / counted bytes) measured on the streaming-copy kernel in the
same run, so unit conventions of FETCH_SIZE / WRITE_SIZE cancel out.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


# Files that hold each profiled kernel's device code and its launch; a
# summary stays valid while these are unchanged.  Other kernels: every file.
KERNEL_SOURCES = {
    "k_bfs_persistent": ["bfs.hip", "bfs_kernels.h", "common.h"],
    "k_msbfs": ["msbfs.hip", "bfs_kernels.h", "common.h"],
}


def kernel_source_hash(kernel: str | None = None) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    files = KERNEL_SOURCES.get(kernel) if kernel else None
    for f in sorted(files or os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def hash_line(kernels) -> str:
    return "# kernel-source hashes: " + ", ".join(f"{k}={kernel_source_hash(k)}" for k in kernels)


def short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {args.cmd}",
             hash_line(args.kernel or ["k_bfs_persistent", "k_msbfs"]) + f", all sources={kernel_source_hash()}", "",
             f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total%':>7s}"]
    for r in rows[:25]:
        lines.append(f"{short(r['Name'])[:60]:60s} {int(r['Calls']):7d} {float(r['AverageNs'])/1e3:10.2f} "
                     f"{float(r['MinNs'])/1e3:10.2f} {float(r['MaxNs'])/1e3:10.2f} {float(r['Percentage']):7.2f}")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_per_dispatch(path, counter):
    """{kernel short name: [value per dispatch]} for one counter."""
    out = {}
    rows = list(csv.DictReader(open(path)))
    by_disp = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Dispatch_Id"], short(r["Kernel_Name"]))
        by_disp[key] = by_disp.get(key, 0.0) + float(r["Counter_Value"])
    for (d, k), v in by_disp.items():
        out.setdefault(k, []).append(v)
    return out


def traffic(args):
    f = _counter_per_dispatch(args.fetch_csv, "FETCH_SIZE")
    w = _counter_per_dispatch(args.write_csv, "WRITE_SIZE")

    def pick(d, sub):
        ks = [k for k in d if sub in k]
        if not ks:
            raise SystemExit(f"no dispatches of {sub} in the counter output")
        vals = [v for k in ks for v in d[k]]
        return sum(vals) / len(vals), len(vals)

    copy_f, _ = pick(f, "k_stream_copy")
    copy_w, _ = pick(w, "k_stream_copy")
    # the copy kernel reads and writes copy_bytes each
    f_scale = args.copy_bytes / copy_f
    w_scale = args.copy_bytes / copy_w
    kf, nf = pick(f, args.kernel)
    kw, nw = pick(w, args.kernel)
    res = {
        "kernel": args.kernel,
        "command": args.cmd,
        "source_hash": kernel_source_hash(args.kernel),
        "dispatches": {"fetch": nf, "write": nw},
        "raw_fetch_per_launch": kf, "raw_write_per_launch": kw,
        "copy_bytes": args.copy_bytes,
        "raw_copy_fetch": copy_f, "raw_copy_write": copy_w,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "fetch_bytes_per_launch": kf * f_scale,
        "write_bytes_per_launch": kw * w_scale,
        "bytes_per_launch": kf * f_scale + kw * w_scale,
    }
    json.dump(res, open(args.out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def counters(args):
    """Average of every collected counter per dispatch of each kernel, and
    the L2 hit rate where TCC_HIT_sum and TCC_MISS_sum were collected."""
    per = {}  # kernel -> counter -> [per-dispatch values]
    for path in args.csv:
        rows = list(csv.DictReader(open(path)))
        names = sorted({r["Counter_Name"] for r in rows})
        for c in names:
            for k, vals in _counter_per_dispatch(path, c).items():
                per.setdefault(k, {})[c] = vals
    lines = ["# rocprofv3 counters, average per dispatch", f"# command: {args.cmd}",
             hash_line([k for k in args.kernel if k in KERNEL_SOURCES]), ""]
    for want in args.kernel:
        ks = [k for k in per if want in k]
        for k in ks:
            lines.append(f"{k}")
            cs = per[k]
            for c in sorted(cs):
                v = cs[c]
                lines.append(f"  {c:28s} {sum(v) / len(v):16.1f}   ({len(v)} dispatches)")
            if "TCC_HIT_sum" in cs and "TCC_MISS_sum" in cs:
                h = sum(cs["TCC_HIT_sum"]) / len(cs["TCC_HIT_sum"])
                m = sum(cs["TCC_MISS_sum"]) / len(cs["TCC_MISS_sum"])
                lines.append(f"  {'L2 hit rate':28s} {h / max(h + m, 1.0):16.3f}")
            lines.append("")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", default="")
    s.add_argument("--kernel", action="append", default=[])
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--kernel", default="k_bfs_persistent")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--cmd", default="")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--out", required=True)
    c.add_argument("--kernel", action="append", default=[])
    c.add_argument("--cmd", default="")
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[a.what](a)


if __name__ == "__main__":
    main()
