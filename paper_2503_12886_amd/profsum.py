"""Summaries of rocprofv3 output for the library's kernels.

Two reports, both from rocprofv3's CSV output (``--output-format csv``):

* ``stats DIR [--window KERNEL:FIRST:COUNT]``: the per-kernel table of a
  ``--kernel-trace --stats`` run (calls, average / min / max duration, share
  of GPU time), short names; with ``--window``, also the average duration of
  one kernel over a range of its launches (a benchmark's timed region);
* ``traffic --fetch DIR --write DIR --kernel NAME --copy-bytes N``: HBM bytes
  per launch of one kernel from two ``--pmc`` passes (``FETCH_SIZE``, then
  ``WRITE_SIZE``, KiB per dispatch summed over counter instances), each scaled
  by what the same counter reads for a plain device-to-device copy of N bytes
  in the same run (the copy reads N and writes N bytes).  With ``--json`` it
  also writes the per-launch bytes, the factors and a hash of the kernel's
  source files, so a reader can tell when the figure went stale; with
  ``--window FIRST:COUNT`` only those launches of the kernel are averaged;
* ``counters DIR [--kernels A,B] [--window KERNEL:FIRST:COUNT ...]``: every
  counter of a ``--pmc`` run, summed over counter instances and averaged per
  dispatch, one row per kernel (a window restricts that kernel's average to
  those launches).

Usage:
  python -m paper_2503_12886_amd.profsum stats out/stats --window composite_bwd:24:100
  python -m paper_2503_12886_amd.profsum traffic --fetch D1 --write D2 \
      --kernel composite_bwd --copy-bytes 268435456 --json profiles/x.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# source files whose change invalidates a kernel's measured traffic
KERNEL_SOURCES = {
    "composite_bwd": ["paper_2503_12886_amd/csrc/raster_bwd.hip", "paper_2503_12886_amd/csrc/gbr_internal.h"],
    "composite_fwd": ["paper_2503_12886_amd/csrc/raster_fwd.hip", "paper_2503_12886_amd/csrc/gbr_internal.h"],
}


def short_name(name: str) -> str:
    """Kernel symbol without namespace, template arguments or parameter list."""
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    n = re.sub(r"<.*>", "", n)
    n = n.replace("void ", "").strip()
    return n.split("::")[-1]


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def _rows(path: str):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats(d: str, top: int = 40) -> str:
    rows = _rows(_find(d, "kernel_stats.csv"))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    agg = collections.OrderedDict()
    for r in rows:
        k = short_name(r["Name"])
        a = agg.setdefault(k, [0, 0.0, float("inf"), 0.0])
        calls = int(r["Calls"])
        a[0] += calls
        a[1] += float(r["TotalDurationNs"])
        a[2] = min(a[2], float(r["MinNs"]))
        a[3] = max(a[3], float(r["MaxNs"]))
    out = [f"{'kernel':40s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for k, (n, t, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{k:40s} {n:7d} {t / n / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} {t / 1e6:10.3f} "
                   f"{100 * t / total:6.2f}")
    return "\n".join(out)


def window(d: str, kernel: str, first: int, count: int) -> str:
    """Average duration of launches first .. first+count-1 (in dispatch order)
    of one kernel, from the per-dispatch kernel trace."""
    rows = [r for r in _rows(_find(d, "kernel_trace.csv")) if short_name(r["Kernel_Name"]).startswith(kernel)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = rows[first:first + count]
    if len(sel) != count:
        raise LookupError(f"{kernel}: {len(rows)} launches traced, window {first}+{count}")
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
    return (f"{kernel} launches {first}..{first + count - 1} of {len(rows)}: avg {sum(dur) / count:.2f} us, "
            f"min {min(dur):.2f} us, max {max(dur):.2f} us")


def _per_dispatch(d: str, counter: str):
    """{dispatch id: (short kernel name, counter value summed over instances)}."""
    rows = _rows(_find(d, "counter_collection.csv"))
    val = collections.defaultdict(float)
    name = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = r["Dispatch_Id"]
        val[k] += float(r["Counter_Value"])
        name[k] = r["Kernel_Name"]
    return {k: (name[k], v) for k, v in val.items()}


def _mean_for(disp, match, win=None) -> tuple:
    vals = [disp[k][1] for k in sorted(disp, key=int) if match(disp[k][0])]
    if win is not None:
        first, count = win
        if len(vals) < first + count:
            raise LookupError(f"{len(vals)} dispatches matched, window {first}+{count}")
        vals = vals[first:first + count]
    if not vals:
        raise LookupError("no dispatch matched")
    return sum(vals) / len(vals), len(vals)


def counters(d: str, kernels=None, windows=None) -> str:
    """Markdown table: kernel, dispatches averaged, then each counter's mean
    per dispatch (summed over its instances)."""
    rows = _rows(_find(d, "counter_collection.csv"))
    names = sorted({r["Counter_Name"] for r in rows})
    per = collections.defaultdict(lambda: collections.defaultdict(float))   # dispatch -> counter -> value
    kname = {}
    for r in rows:
        per[r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
        kname[r["Dispatch_Id"]] = short_name(r["Kernel_Name"])
    by_kernel = collections.defaultdict(list)
    for k in sorted(per, key=int):
        by_kernel[kname[k]].append(per[k])
    windows = windows or {}
    out = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for kn in sorted(by_kernel):
        if kernels and not any(kn.startswith(x) for x in kernels):
            continue
        v = by_kernel[kn]
        w = next((windows[x] for x in windows if kn.startswith(x)), None)
        if w is not None:
            v = v[w[0]:w[0] + w[1]]
        if not v:
            continue
        cells = [f"{sum(x[c] for x in v) / len(v):.4g}" for c in names]
        out.append(f"| {kn} | {len(v)} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int, copy_match: str, win=None):
    fetch = _per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _per_dispatch(write_dir, "WRITE_SIZE")

    def is_kernel(n):
        return short_name(n).startswith(kernel)

    def is_copy(n):
        return copy_match.lower() in n.lower()

    kib = 1024.0
    f_k, nf = _mean_for(fetch, is_kernel, win)
    w_k, nw = _mean_for(write, is_kernel, win)
    # the copy of known size: the largest matching dispatch in each pass
    f_c = max(v for (n, v) in fetch.values() if is_copy(n))
    w_c = max(v for (n, v) in write.values() if is_copy(n))
    ff = copy_bytes / (f_c * kib)
    fw = copy_bytes / (w_c * kib)
    res = {"kernel": kernel, "launches": [nf, nw], "window": list(win) if win else None,
           "fetch_kib_raw": f_k, "write_kib_raw": w_k,
           "copy_bytes": copy_bytes, "copy_fetch_kib_raw": f_c, "copy_write_kib_raw": w_c,
           "fetch_factor": ff, "write_factor": fw,
           "fetch_bytes_per_launch": f_k * kib * ff, "write_bytes_per_launch": w_k * kib * fw}
    res["bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    others = collections.defaultdict(list)
    for (n, v) in fetch.values():
        others[short_name(n)].append(v)
    res["fetch_kib_by_kernel"] = {k: sum(v) / len(v) for k, v in sorted(others.items())}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=40)
    s.add_argument("--window", help="KERNEL:FIRST:COUNT, the average over those launches of KERNEL "
                                    "(a benchmark's timed region) from the kernel trace")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--copy-match", default="copy")
    t.add_argument("--json")
    t.add_argument("--window", help="FIRST:COUNT, average over those launches of the kernel only")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernels", help="comma-separated name prefixes")
    c.add_argument("--window", action="append", default=[], help="KERNEL:FIRST:COUNT (repeatable)")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        wins = {}
        for w in a.window:
            k, first, count = w.split(":")
            wins[k] = (int(first), int(count))
        print(counters(a.dir, a.kernels.split(",") if a.kernels else None, wins))
        return 0
    if a.cmd == "stats":
        print(stats(a.dir, a.top))
        if a.window:
            k, first, count = a.window.split(":")
            print(window(a.dir, k, int(first), int(count)))
        return 0
    win = tuple(int(x) for x in a.window.split(":")) if a.window else None
    res = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.copy_match, win)
    if a.json:
        srcs = KERNEL_SOURCES.get(a.kernel, [])
        meta = dict(res, sources=srcs, source_hash=source_hash(srcs))
        with open(a.json, "w") as fh:
            json.dump(meta, fh, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "fetch_kib_by_kernel"}, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
