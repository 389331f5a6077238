"""Summaries of rocprofv3 CSV output for the benchmark's kernels.

    python -m paper_1706_06750_amd.rocprof_summary stats  <kernel_stats.csv>
    python -m paper_1706_06750_amd.rocprof_summary traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> --workload NAME --pixels P --copy-mib M --out <json>

``stats`` prints the kernel-duration table.  ``traffic`` turns FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) into HBM bytes per step of the level segment:
each counter is scaled by what it reads for the library's copy kernel, which
moves a known number of bytes (M MiB read and M MiB written); for every AOS
launch shape that ran, the bytes of one dispatch of each of its three
kernels are summed, and the detector's bytes per level are kept apart (a
run with d detector levels inside its segment adds d / 15 of them per
step).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

AOS_KERNELS = ("aos_reduce_kernel", "aos_iface_kernel", "aos_recover_kernel")
# recovery kernels by name (two lanes per chunk, or one), counted as one role
RECOVER_NAMES = ("aos_recover_kernel", "aos_recover_split_kernel")


def base_name(name: str) -> str:
    """Kernel name without template arguments, the recovery variants under
    aos_recover_kernel."""
    base = name.split("<")[0]
    return "aos_recover_kernel" if base in RECOVER_NAMES else base
DET_KERNELS = ("det_strip_kernel",)


def short(name: str) -> str:
    """'void kaze::(anonymous namespace)::det_strip_kernel<2, 3>(kaze::BatchImage, ...)'
    -> 'det_strip_kernel<2, 3>'."""
    n = name.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):   # cut at the parameter list (outside <...>)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    return n.split("::")[-1] if "<" not in n else n[n.rfind("::", 0, n.find("<")) + 2:]


# Sources of the per-level kernels: a change to any of them invalidates a
# traffic summary.
LEVEL_SOURCES = ("aos.hip", "tile_stage.h", "kaze_internal.h", "detect.hip")


def csrc_hash(root: str) -> str:
    h = hashlib.sha256()
    d = os.path.join(root, "paper_1706_06750_amd", "csrc")
    for f in LEVEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append("| %s | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def parse_shape(label: str):
    """'60x32 c30/32 m4' -> (tile height, row chunk, column chunk, interface
    chunks per lane) as strings."""
    tile, chunks, m = label.split()
    rc, cc = chunks[1:].split("/")
    return tile.split("x")[1], rc, cc, m[1:]


def template_args(name: str):
    return [a.strip() for a in name.split("<", 1)[1].rsplit(">", 1)[0].split(",")]


def _rows(path: str, counter: str):
    """Rows of one counter in dispatch order."""
    rows = [r for r in csv.DictReader(open(path))
            if r.get("Counter_Name", r.get("counter_name")) == counter]
    rows.sort(key=lambda r: int(r.get("Dispatch_Id", r.get("dispatch_id", 0))))
    return rows


def counter_means(path: str, counter: str, aos_shape: str | None = None):
    """Mean counter value per dispatch, by kernel.  With aos_shape (a shape
    label, '60x32 c30/32 m4') only the AOS kernels of that shape count (the
    autotuner runs every shape first): aos_reduce_kernel<RG, TY, RC, CC, CG,
    GM>, aos_recover(_split)_kernel<TY, RC, CC>, and aos_iface_kernel<M> dispatches
    whose preceding reduction (in dispatch order) had that shape's tile."""
    acc = collections.defaultdict(list)
    want = parse_shape(aos_shape) if aos_shape else None
    last_tile = None
    for r in _rows(path, counter):
        name = short(r.get("Kernel_Name", r.get("kernel_name")))
        base = base_name(name)
        if base == "aos_reduce_kernel":
            last_tile = tuple(template_args(name)[1:4])
        if want and base == "aos_reduce_kernel" and last_tile != want[:3]:
            continue
        if want and base == "aos_recover_kernel" and tuple(template_args(name)) != want[:3]:
            continue
        if want and base == "aos_iface_kernel" and (template_args(name)[0] != want[3] or
                                                    last_tile != want[:3]):
            continue
        acc[base].append(float(r.get("Counter_Value", r.get("value"))))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def counter_totals(path: str, counter: str):
    """Sum of the counter over every dispatch and number of dispatches, by
    kernel (all template instances together)."""
    tot = collections.defaultdict(float)
    cnt = collections.defaultdict(int)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        base = base_name(short(r.get("Kernel_Name", r.get("kernel_name"))))
        tot[base] += float(r.get("Counter_Value", r.get("value")))
        cnt[base] += 1
    return tot, cnt


def shapes_present(path: str, counter: str):
    """Launch-shape labels ('60x32 c30/32 m4') whose three AOS kernels all
    appear in the counter file: reduction and recovery (tile height, chunk
    lengths) crossed with the interface solve's chunks per lane."""
    tiles, ms = set(), set()
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = short(r.get("Kernel_Name", r.get("kernel_name")))
        base = base_name(name)
        if base == "aos_recover_kernel":
            tiles.add(tuple(template_args(name)))
        elif base == "aos_iface_kernel":
            ms.add(template_args(name)[0])
    return sorted("60x%s c%s/%s m%s" % (ty, rc, cc, m) for ty, rc, cc in tiles for m in ms)


def traffic(fetch_csv, write_csv, copy_mib, root, workload, pixels, levels=16):
    """HBM bytes per step of the level segment, for every AOS launch shape
    that ran (the autotuner runs each): the AOS kernels' mean dispatch of
    that shape; and the detector's bytes per level (every run holds
    levels - 1 reductions, whatever the shape), to add for the detector
    levels that run inside the segment."""
    known_kib = copy_mib * 1024.0
    f_all = counter_means(fetch_csv, "FETCH_SIZE")
    w_all = counter_means(write_csv, "WRITE_SIZE")
    fs = known_kib / f_all["copy_kernel"]
    ws = known_kib / w_all["copy_kernel"]
    by_shape = {}
    for label in shapes_present(fetch_csv, "FETCH_SIZE"):
        f = counter_means(fetch_csv, "FETCH_SIZE", label)
        w = counter_means(write_csv, "WRITE_SIZE", label)
        if not all(k in f and k in w for k in AOS_KERNELS):
            continue
        per = {k: {"fetch_kib_raw": f[k], "write_kib_raw": w[k],
                   "bytes": (f[k] * fs + w[k] * ws) * 1024.0} for k in AOS_KERNELS}
        total = sum(v["bytes"] for v in per.values())
        by_shape[label] = {"kernels": per, "bytes": total, "bytes_per_pixel": total / pixels}
    det = None
    ft, fc = counter_totals(fetch_csv, "FETCH_SIZE")
    wt, wc = counter_totals(write_csv, "WRITE_SIZE")
    if any(ft.get(k) for k in DET_KERNELS):
        runs_f = fc["aos_reduce_kernel"] / (levels - 1)
        runs_w = wc["aos_reduce_kernel"] / (levels - 1)
        fk = sum(ft.get(k, 0.0) for k in DET_KERNELS) / runs_f / levels
        wk = sum(wt.get(k, 0.0) for k in DET_KERNELS) / runs_w / levels
        det = {"fetch_kib_raw": fk, "write_kib_raw": wk, "bytes": (fk * fs + wk * ws) * 1024.0,
               "bytes_per_pixel": (fk * fs + wk * ws) * 1024.0 / pixels}
    return {"workload": workload, "pixels": pixels, "levels": levels,
            "copy_scale_fetch": fs, "copy_scale_write": ws,
            "aos_by_shape": by_shape, "det_per_level": det, "csrc_hash": csrc_hash(root)}


def segment_bytes(d: dict, aos_tile: str, det_levels: int):
    """Bytes per step of the level segment from a traffic summary: the shape's
    AOS kernels plus det_levels / (levels - 1) detector levels; None when the
    shape or (det_levels > 0) the detector did not run in the profile."""
    a = d["aos_by_shape"].get(aos_tile)
    if a is None or (det_levels and d.get("det_per_level") is None):
        return None
    det = d["det_per_level"]["bytes"] if det_levels else 0.0
    return a["bytes"] + det_levels / (d["levels"] - 1) * det


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--workload", required=True, help="workload name, e.g. 1920x1200")
    b.add_argument("--pixels", type=int, required=True, help="pixels per level of one run")
    b.add_argument("--copy-mib", type=int, required=True)
    b.add_argument("--out", required=True)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if args.cmd == "stats":
        print(stats(args.csv))
    else:
        d = traffic(args.fetch_csv, args.write_csv, args.copy_mib, root, args.workload,
                    args.pixels)
        with open(args.out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
