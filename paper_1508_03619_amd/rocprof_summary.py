"""Summarise rocprofv3 output for the committed profiles.

Usage:
  python -m paper_1508_03619_amd.rocprof_summary stats <kernel_stats.csv> <out.txt> --cmd "<command>"
  python -m paper_1508_03619_amd.rocprof_summary traffic <fetch_counter_collection.csv>
         <write_counter_collection.csv> <out.json> --kernel k_bfs_persistent --copy-bytes N --cmd "..."
  python -m paper_1508_03619_amd.rocprof_summary counters <counter_collection.csv>... --out <out.txt>
         --kernel k_bfs_persistent --kernel k_msbfs --cmd "..."
  python -m paper_1508_03619_amd.rocprof_summary levels <fetch.csv> <write.csv> <bench log> <out.txt>
         --copy-bytes N --cmd "..."

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


def _dispatches(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _copy_scale(rows, copy_bytes):
    v = [float(r["Counter_Value"]) for r in rows if "k_stream_copy" in r["Kernel_Name"]]
    return copy_bytes / (sum(v) / len(v))


def _searches(rows):
    """Groups the per-level schedule's dispatches into searches: k_dd_init,
    then (k_dd_convert, k_dd_step, k_dd_publish) per level, then k_dd_fixup.
    Returns the searches run without statistics, each as a dict of
    (fetch-or-write value, duration ns) lists."""
    out, cur = [], None
    for r in rows:
        k = r["Kernel_Name"]
        if "k_dd_" not in k:
            continue
        v = float(r["Counter_Value"])
        t = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if "k_dd_init" in k:
            cur = {"init": (v, t), "convert": [], "step": [], "publish": [], "fixup": None, "stats": False}
            out.append(cur)
        elif cur is None:
            continue
        elif "k_dd_convert" in k:
            cur["convert"].append((v, t))
        elif "k_dd_step" in k:
            cur["step"].append((v, t))
            cur["stats"] = cur["stats"] or "<true>" in k
        elif "k_dd_publish" in k:
            cur["publish"].append((v, t))
        elif "k_dd_fixup" in k:
            cur["fixup"] = (v, t)
    return [s for s in out if not s["stats"] and s["fixup"] is not None]


def level_alg_bytes(rec, prev_dir, n):
    """Algorithmic bytes of one level record [direction, frontier,
    frontier_edges, claimed, scanned, unvisited] (the search's byte model):
    returns (bytes of the step, bytes of the conversion before it)."""
    d, f, mf, cl, sc, un = rec
    if d == 1:
        conv = 20 * f + n // 8 if prev_dir == 2 else 0
        return 20 * f + 8 * mf + 12 * cl, conv
    conv = 4 * f + n // 8 if prev_dir == 1 else 0
    return 16 * un + 4 * sc + 3 * n // 8 + 8 * cl, conv


def levels(args):
    """Per-level attribution of FETCH_SIZE / WRITE_SIZE and time for the
    per-level schedule (one launch per step)."""
    recs = [json.loads(l[len("LEVELS "):]) for l in open(args.log) if l.startswith("LEVELS ")]
    F, W = _dispatches(args.fetch), _dispatches(args.write)
    fs, ws = _copy_scale(F, args.copy_bytes), _copy_scale(W, args.copy_bytes)
    sf, sw = _searches(F), _searches(W)
    if not (len(sf) == len(sw) == len(recs)):
        raise SystemExit(f"{len(sf)} fetch searches, {len(sw)} write searches, {len(recs)} records")
    cats = {}

    def add(cat, fv, wv, t, alg):
        c = cats.setdefault(cat, [0, 0.0, 0.0, 0, 0])
        c[0] += 1
        c[1] += fv * fs
        c[2] += wv * ws
        c[3] += t
        c[4] += alg

    for s_f, s_w, rec in zip(sf, sw, recs):
        n = rec["n"]
        g = rec["graph"]
        lv = rec["levels"]
        if len(s_f["step"]) != len(lv):
            raise SystemExit(f"{g} source {rec['source']}: {len(s_f['step'])} steps, {len(lv)} records")
        add(f"{g} init", s_f["init"][0], s_w["init"][0], s_f["init"][1], 16 * n + 8)
        prev, first_bu = 1, True
        for i, r in enumerate(lv):
            step_alg, conv_alg = level_alg_bytes(r, prev, n)
            if r[0] == 1:
                cat = f"{g} top-down, m_f <= 32768" if r[2] <= 32768 else f"{g} top-down, m_f > 32768"
            else:
                cat = f"{g} bottom-up, first" if first_bu else f"{g} bottom-up, later"
                first_bu = False
            add(cat, s_f["step"][i][0], s_w["step"][i][0], s_f["step"][i][1], step_alg)
            if conv_alg:
                add(f"{g} conversion", s_f["convert"][i][0], s_w["convert"][i][0], s_f["convert"][i][1], conv_alg)
            add(f"{g} level boundary (publish)", s_f["publish"][i][0], s_w["publish"][i][0], s_f["publish"][i][1], 0)
            prev = r[0]
        add(f"{g} final pass", s_f["fixup"][0], s_w["fixup"][0], s_f["fixup"][1], 8 * n)
    lines = ["# per-level attribution of counted traffic and time, per-level schedule (mode 1)",
             f"# command: {args.cmd}", hash_line(["k_bfs_persistent"]),
             f"# {len(recs)} searches; fetch scale {fs:.1f} B/unit, write scale {ws:.1f} B/unit (copy kernel)",
             "# columns are per occurrence: MB fetched, MB written, algorithmic MB, counted/algorithmic, us",
             "", f"{'category':44s} {'count':>5s} {'fetch MB':>9s} {'write MB':>9s} {'alg MB':>8s} "
             f"{'ratio':>6s} {'us':>8s}"]
    for cat in sorted(cats):
        c, fb, wb, t, alg = cats[cat]
        ratio = (fb + wb) / alg if alg else float("nan")
        lines.append(f"{cat:44s} {c:5d} {fb / c / 1e6:9.2f} {wb / c / 1e6:9.2f} {alg / c / 1e6:8.2f} "
                     f"{ratio:6.2f} {t / c / 1e3:8.1f}")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    lv = sub.add_parser("levels")
    lv.add_argument("fetch")
    lv.add_argument("write")
    lv.add_argument("log", help="bench.py --profile-levels output (its LEVELS lines)")
    lv.add_argument("out")
    lv.add_argument("--copy-bytes", type=float, required=True)
    lv.add_argument("--cmd", default="")
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters, "levels": levels}[a.what](a)


if __name__ == "__main__":
    main()
