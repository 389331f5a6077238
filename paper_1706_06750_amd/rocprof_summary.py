"""Summaries of rocprofv3 CSV output for the benchmark's kernels.

    python -m paper_1706_06750_amd.rocprof_summary stats  <kernel_stats.csv>
    python -m paper_1706_06750_amd.rocprof_summary traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> --image WxH --copy-mib M --out <json>

``stats`` prints the kernel-duration table.  ``traffic`` turns FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) into HBM bytes per step of the level segment:
each counter is scaled by what it reads for the library's copy kernel, which
moves a known number of bytes (M MiB read and M MiB written); the bytes of
one dispatch of each AOS kernel are summed, plus those of one detector
dispatch (one level) times 16/15 (16 detector levels per 15 steps).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

AOS_KERNELS = ("aos_reduce_kernel", "aos_iface_kernel", "aos_recover_kernel")
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


def counter_means(path: str, counter: str, aos_shape: str | None = None):
    """Mean counter value per dispatch, by kernel.  With aos_shape (a shape
    label, '60x32 c30/32 m4') only the AOS kernels instantiated for that
    shape count (the autotuner runs every shape first):
    aos_reduce_kernel<RG, TY, RC, CC, CG, GM>, aos_iface_kernel<M>,
    aos_recover_kernel<TY, RC, CC>."""
    acc = collections.defaultdict(list)
    want = parse_shape(aos_shape) if aos_shape else None
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = short(r.get("Kernel_Name", r.get("kernel_name")))
        base = name.split("<")[0]
        if want and base == "aos_reduce_kernel" and tuple(template_args(name)[1:4]) != want[:3]:
            continue
        if want and base == "aos_recover_kernel" and tuple(template_args(name)) != want[:3]:
            continue
        if want and base == "aos_iface_kernel" and template_args(name)[0] != want[3]:
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
        base = short(r.get("Kernel_Name", r.get("kernel_name"))).split("<")[0]
        tot[base] += float(r.get("Counter_Value", r.get("value")))
        cnt[base] += 1
    return tot, cnt


def traffic(fetch_csv, write_csv, W, H, copy_mib, root, aos_tile, det_levels=0, pixels=0,
            levels=16):
    """Bytes per step of the level segment: the AOS kernels' mean dispatch
    (the chosen launch shape only) plus, when det_levels detector levels run inside
    the segment, their share: the detector's bytes per run (every run holds
    levels - 1 reductions, whatever the shape) / levels * det_levels, spread
    over the levels - 1 steps."""
    f = counter_means(fetch_csv, "FETCH_SIZE", aos_tile)
    w = counter_means(write_csv, "WRITE_SIZE", aos_tile)
    known_kib = copy_mib * 1024.0
    fs = known_kib / f["copy_kernel"]
    ws = known_kib / w["copy_kernel"]
    per = {}
    for k in AOS_KERNELS:
        per[k] = {"fetch_kib_raw": f[k], "write_kib_raw": w[k],
                  "bytes": (f[k] * fs + w[k] * ws) * 1024.0}
    if det_levels:
        ft, fc = counter_totals(fetch_csv, "FETCH_SIZE")
        wt, wc = counter_totals(write_csv, "WRITE_SIZE")
        runs_f = fc["aos_reduce_kernel"] / (levels - 1)
        runs_w = wc["aos_reduce_kernel"] / (levels - 1)
        fk = sum(ft[k] for k in DET_KERNELS) / runs_f / levels
        wk = sum(wt[k] for k in DET_KERNELS) / runs_w / levels
        share = det_levels / (levels - 1)
        per["det (%d levels in the segment)" % det_levels] = {
            "fetch_kib_raw_per_level": fk, "write_kib_raw_per_level": wk,
            "bytes": share * (fk * fs + wk * ws) * 1024.0}
    total = sum(v["bytes"] for v in per.values())
    return {"image": "%dx%d" % (W, H) if W else None, "aos_tile": aos_tile,
            "det_levels_in_segment": det_levels,
            "copy_scale_fetch": fs, "copy_scale_write": ws,
            "kernels": per, "bytes_per_level": total,
            "pixels": pixels or W * H,
            "bytes_per_pixel_level": total / (pixels or W * H), "csrc_hash": csrc_hash(root)}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--image", required=True, help="WxH of the single image, or a workload name")
    b.add_argument("--copy-mib", type=int, required=True)
    b.add_argument("--aos-tile", required=True,
                   help="AOS launch shape of the run, e.g. '60x32 c30/32 m4'")
    b.add_argument("--det-levels", type=int, default=0,
                   help="detector levels that run inside the level segment (the batch's "
                        "det_levels_in_segment property)")
    b.add_argument("--pixels", type=int, default=0,
                   help="pixels per level when the run covers several images (default W*H)")
    b.add_argument("--out", required=True)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if args.cmd == "stats":
        print(stats(args.csv))
    else:
        W, H = (int(v) for v in args.image.split("x")) if "x" in args.image else (0, 0)
        d = traffic(args.fetch_csv, args.write_csv, W, H, args.copy_mib, root, args.aos_tile,
                    args.det_levels, args.pixels)
        with open(args.out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
