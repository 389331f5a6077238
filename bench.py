"""Throughput benchmark: KAZE scale space + detector response + extrema.

One step = one 1920x1200 synthetic image (already resident in HBM) through
the whole plain path: Gaussian pre-smoothing, contrast factor, 15 levels of
conductivity + AOS step, the Hessian determinant of all 16 levels and the
3x3x3 extrema.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1920x1200 scale-space+Hessian images/s, AOS vs surrogate; % HBM peak"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense MFMA, MI355X
# the middle pair of the surrogate's layers (two 32 -> 32 convolutions in one
# launch): 2 * 2 * 32 * 32 * 9 FLOP per pixel
CONV_FLOP_PER_PX = 2 * 2 * 32 * 32 * 9
# The dominant work is the level segment of a run: 15 levels of conductivity
# and AOS step (aos_reduce computes g and reduces every chunk, aos_iface
# solves the interface systems, aos_recover recovers the chunks and
# averages), with the detector response of each of the 16 levels running on
# a second stream beside the later steps.  Algorithmic HBM bytes per pixel:
# conductivity reads L_{i-1} and writes g (8), the AOS step reads L_{i-1}
# and g and writes L_i (12), the detector reads L_i and writes det_i (8).
STEP_ALGO_BYTES_PER_PX = 20
DET_ALGO_BYTES_PER_PX = 8
AOS_KERNELS = ("aos_reduce", "aos_iface", "aos_recover")


def tile_label(K, shape):
    """Tile, chunk lengths and interface lanes of an AOS launch shape, e.g.
    '60x32 c30/32 m4'."""
    return K.shape_label(shape)


def traffic_from_profile(key, aos_tile, det_levels):
    """HBM bytes per step of the level segment from the committed counter
    summary profiles/level_traffic_<key>.json, if it was taken on the current
    per-level kernel sources: the chosen launch shape's AOS kernels plus the
    detector levels that run inside the segment."""
    from paper_1706_06750_amd.rocprof_summary import csrc_hash, segment_bytes
    path = os.path.join(ROOT, "profiles", "level_traffic_%s.json" % key)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("csrc_hash") != csrc_hash(ROOT) or "aos_by_shape" not in d:
        return None
    b = segment_bytes(d, aos_tile, det_levels)
    return None if b is None else round(b)


CPU_BASELINE_SRC = r"""
import sys, time, json
sys.path.insert(0, %r)
import numpy as np
import oracle as O
from synthetic import kaze_image
W, H, seeds = %d, %d, %r
imgs = [kaze_image(W, H, s).astype(np.float64) for s in seeds]
t = time.perf_counter()
for img in imgs:
    lev, k = O.build_scale_space(img)
    det = O.detector_response(lev)
    kp = O.find_extrema(det, 0.001)
print(json.dumps({"seconds": time.perf_counter() - t, "images": len(imgs)}))
"""

CPU_BASELINE_PER_PROCESS = 2  # images per worker: about 8-10 s of work each


def cpu_baseline(W, H, seed):
    """The FP64 oracle as it stands on the host: P single-threaded worker
    processes (P = the cores this process may use, at most 16: the host's CPU
    share of one GPU on an eight-GPU machine), each running
    the full path on CPU_BASELINE_PER_PROCESS images of the workload's size
    (seeds seed, seed + 1, ...), all started together; throughput = images /
    wall time of the slowest worker (imports and input generation outside
    the timed part)."""
    affinity = len(os.sched_getaffinity(0))
    P = max(1, min(16, affinity))
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[v] = "1"
    procs = []
    for w in range(P):
        seeds = [seed + w * CPU_BASELINE_PER_PROCESS + i for i in range(CPU_BASELINE_PER_PROCESS)]
        procs.append(subprocess.Popen([sys.executable, "-c", CPU_BASELINE_SRC % (ROOT, W, H, seeds)],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                                      env=env))
    secs = []
    for pr in procs:
        out, err = pr.communicate(timeout=900)
        if pr.returncode != 0:
            raise RuntimeError("oracle baseline failed: " + err[-2000:])
        secs.append(json.loads(out.strip().splitlines()[-1])["seconds"])
    n = P * CPU_BASELINE_PER_PROCESS
    return {"value": n / max(secs), "unit": "images/s", "cores": P, "kind": "oracle",
            "host_cores": os.cpu_count(), "affinity_cores": affinity,
            "sample": "%d images %dx%d (seeds %d..%d), full path: scale space, det, extrema; "
                      "%d single-threaded processes, %.1f s each (slowest %.1f s); one image "
                      "on one core %.2f s" % (n, W, H, seed, seed + n - 1, P,
                                              sum(secs) / P, max(secs),
                                              min(secs) / CPU_BASELINE_PER_PROCESS)}


def level_roofline(level_us, px, traffic, levels=16, det_levels=0):
    """Per step of the level segment (its time / (levels - 1)); algorithmic
    bytes of the segment (the steps and the detector levels that run beside
    them) spread over the steps."""
    seg = (levels - 1) * STEP_ALGO_BYTES_PER_PX + det_levels * DET_ALGO_BYTES_PER_PX
    algo = seg * px / (levels - 1)
    achieved = algo / (level_us * 1e-6) / 1e9
    return {
        "kernel": "one level of the level segment: conductivity + AOS step (" +
                  "+".join(AOS_KERNELS) + ")" +
                  (" with the detector of %d levels overlapped" % det_levels if det_levels else ""),
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": algo,
        "us_per_launch": round(level_us, 3),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kaze_1920x1200")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate measurements (plain path only)")
    ap.add_argument("--no-substeps", action="store_true",
                    help="skip the sub-steps-per-level measurement")
    ap.add_argument("--no-keypoints", action="store_true",
                    help="skip the extrema-window and refinement measurements")
    ap.add_argument("--no-fed", action="store_true",
                    help="skip the FED-scheme measurement")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the per-kernel timing pass (for profiler runs)")
    ap.add_argument("--forms", choices=("both", "eager", "graph"), default="both",
                    help="launch forms of the image and batch plans to time (both: the "
                         "faster is reported)")
    ap.add_argument("--no-batches", action="store_true",
                    help="skip the batch measurements beside the single image (the 64-image "
                         "uneven batch, 8 x 1920x1200, the 4K + 720p surrogate batch)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run the library's copy kernel on this many MiB, a known-size "
                         "reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(images shard across GPUs with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1706_06750_amd import kaze as K
    from synthetic import WORKLOADS, kaze_image

    cases = WORKLOADS[args.workload]()
    torch.cuda.set_device(0)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            K.kaze_copy_f32(src, dst, n)
        torch.cuda.synchronize()
        del src, dst

    if len(cases) == 1:
        rec = bench_single(args, K, torch, kaze_image, cases[0])
    else:
        rec = bench_batch(args, K, torch, kaze_image, cases)
    print(json.dumps(rec), flush=True)


def progress(msg):
    """One line per finished stage on stderr (the JSON record is stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def record(args, value, ms_per_step, config, roofline, extra):
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
    }
    rec.update(extra)
    return rec


def timed_runs(args, K, torch, kb, eager):
    """Timed region: runs of the plan (eager launches or graph replays), each
    followed by the readback of every image's keypoint count into pinned
    host memory (an asynchronous copy on the run's stream); an event pair
    brackets the AOS-step segment of every run on the stream it runs on.
    Returns (seconds, microseconds per level)."""
    counts = torch.empty((max(args.steps, args.warmup), kb.counts.numel()), dtype=torch.int32,
                         pin_memory=True)
    for i in range(args.warmup):
        kb.run(eager=eager)
        counts[i].copy_(kb.counts, non_blocking=True)
    torch.cuda.synchronize()
    K.kaze_profile_begin("aos_reduce")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        kb.run(eager=eager)
        counts[i].copy_(kb.counts, non_blocking=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    runs, ms = K.kaze_profile_end()
    assert runs == args.steps
    if not torch.equal(counts[args.steps - 1], kb.counts.cpu()):
        raise RuntimeError("keypoint counts read back in the timed region disagree")
    return elapsed, 1e3 * ms / (runs * (kb.N - 1))


def run_distribution_and_transfers(args, K, torch, kb, img_cpu, form, reps=50):
    """Outside the timed region: the per-run time distribution of the plan
    (an event pair around every run and its keypoint-count readback, on the
    stream the plan runs on), the upload of the FP32 image from pinned host
    memory and the download of the keypoint list into pinned host memory,
    each timed with event pairs.  The PCIe-inclusive rate adds one upload
    and one download to the median run (no overlap between them)."""
    eager = form == "eager"
    s = torch.cuda.current_stream()
    counts = torch.empty(kb.counts.numel(), dtype=torch.int32, pin_memory=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for _ in range(3):
        kb.run(eager=eager)
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(s)
        kb.run(eager=eager)
        counts.copy_(kb.counts, non_blocking=True)
        b.record(s)
    torch.cuda.synchronize()
    run_us = sorted(1e3 * a.elapsed_time(b) for a, b in ev)

    def pct(v, q):
        return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]

    host = torch.from_numpy(img_cpu).pin_memory()
    up = []
    for _ in range(20):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        kb.inputs[0].copy_(host, non_blocking=True)
        b.record(s)
        torch.cuda.synchronize()
        up.append(1e3 * a.elapsed_time(b))
    kb.run(eager=eager)
    torch.cuda.synchronize()
    n = min(int(kb.count[0].item()), kb.capacity)
    kp_host = torch.empty((max(n, 1), 4), dtype=torch.int32, pin_memory=True)
    down = []
    for _ in range(20):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        kp_host[:n].copy_(kb.kps[0][:n], non_blocking=True)
        b.record(s)
        torch.cuda.synchronize()
        down.append(1e3 * a.elapsed_time(b))
    up_us, down_us = sorted(up)[len(up) // 2], sorted(down)[len(down) // 2]
    med = pct(run_us, 0.5)
    nbytes = img_cpu.nbytes
    return {"per_run_us": {"median": round(med, 2), "p10": round(pct(run_us, 0.1), 2),
                           "p90": round(pct(run_us, 0.9), 2), "runs": reps, "form": form},
            "upload": {"bytes": nbytes, "us": round(up_us, 2),
                       "GB_per_s": round(nbytes / (up_us * 1e-6) / 1e9, 2)},
            "keypoint_download": {"keypoints": n, "bytes": 16 * n, "us": round(down_us, 2)},
            "pcie_inclusive_images_per_s": round(1e6 / (up_us + med + down_us), 2)}


def det_levels_of(kb, form):
    """Detector levels inside the level segment of a run (either launch form):
    all levels for batches that fork the detector beside the steps, else 0."""
    return kb.det_levels_in_segment


def timed_plan(args, K, torch, kb, n_images):
    """Both launch forms of the plan (or the one --forms names) are timed over
    the same K steps; the faster is the reported one.  Returns (seconds, us
    per level, form, the per-form figures)."""
    names = ("eager", "graph") if args.forms == "both" else (args.forms,)
    res = {form: timed_runs(args, K, torch, kb, form == "eager") for form in names}
    best = min(res, key=lambda f: res[f][0])
    forms = {f: {"images_per_s": round(n_images * args.steps / e, 3), "us_per_level": round(u, 3)}
             for f, (e, u) in res.items()}
    return res[best][0], res[best][1], best, forms


def bench_single(args, K, torch, kaze_image, case):
    W, H, seed = case
    img = torch.from_numpy(kaze_image(W, H, seed)).cuda()

    # per-kernel breakdown and eager throughput of the single-image calls
    kz = K.Kaze(W, H)
    for _ in range(args.warmup):
        kz.run(img)
    torch.cuda.synchronize()
    breakdown = {}
    probe_steps = max(5, min(20, args.steps))
    for name in K.kaze_kernel_names():
        if name == "copy" or args.no_breakdown:
            continue
        K.kaze_profile_begin(name)
        for _ in range(probe_steps):
            kz.run(img)
        n, ms = K.kaze_profile_end()
        if n:
            breakdown[name] = {"launches_per_step": n / probe_steps,
                               "ms_per_step": ms / probe_steps, "us_per_launch": 1e3 * ms / n}
    for _ in range(3):
        kz.run(img)
    torch.cuda.synchronize()
    eager_steps = max(50, args.steps)
    t1 = time.perf_counter()
    for _ in range(eager_steps):
        kz.run(img)
    torch.cuda.synchronize()
    eager_value = eager_steps / (time.perf_counter() - t1)

    # timed path: the image's plan (eager launches or graph replays, the
    # faster of the two)
    progress("single-image calls: %.1f images/s" % eager_value)
    kb = K.KazeBatch([(W, H)], shape="auto")
    kb.inputs[0].copy_(img)
    elapsed, level_us, form, forms = timed_plan(args, K, torch, kb, 1)
    progress("image plan: %.1f images/s (%s)" % (args.steps / elapsed, form))
    roof = level_roofline(level_us, W * H,
                          traffic_from_profile("%dx%d" % (W, H), tile_label(K, kb.shape),
                                               det_levels_of(kb, form)),
                          det_levels=det_levels_of(kb, form))
    roof["timed_in"] = "the timed region (event pair around each run's AOS segment)"
    kps = int(kb.count[0].item())
    shape = tile_label(K, kb.shape)
    transfers = run_distribution_and_transfers(args, K, torch, kb, kaze_image(W, H, seed), form)
    kb.close()

    extra = {"eager_images_per_s": round(eager_value, 3), "plan_launch_forms": forms,
             "run_distribution_and_transfers": transfers,
             "kernel_breakdown": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                                  for k, v in breakdown.items()}}
    if not args.no_fed:
        extra["fed"] = bench_fed(args, K, torch, img, W, H, args.steps / elapsed, eager_value)
        progress("FED done")
    if not args.no_keypoints:
        extra["keypoints"] = bench_keypoints(args, K, torch, img, W, H)
        progress("keypoint stages done")
    if not args.no_substeps:
        extra["substeps"] = bench_substeps(args, K, torch, img, W, H, eager_value)
        progress("sub-steps done")
    if not args.no_surrogate:
        extra["surrogate"] = bench_surrogate(args, K, torch, img, W, H, seed,
                                             args.steps / elapsed)
        progress("surrogate done")
    N = kz.N
    if not args.no_batches:
        del img, kz
        torch.cuda.empty_cache()
        extra["batches"] = bench_batches(args, K, torch, kaze_image)
    if not args.no_cpu_baseline:
        extra["cpu_baseline"] = cpu_baseline(W, H, seed)
        progress("CPU baseline: %.3f images/s" % extra["cpu_baseline"]["value"])
    config = {"workload": args.workload, "image": "%dx%d" % (W, H), "seed": seed,
              "levels": N,
              "path": "plain AOS (no surrogate), image plan, %s" %
                      ("eager launches" if form == "eager" else "graph replay"),
              "aos_tile": shape, "keypoints": kps}
    return record(args, args.steps / elapsed, 1e3 * elapsed / args.steps, config, roof, extra)


def bench_fed(args, K, torch, img, W, H, plain_value, plain_eager):
    """The FED scheme (one fast-explicit-diffusion cycle per level) on the
    same image, eager calls: images/s, time per level (conductivity + cycle,
    event pairs around every launch) and the cycle lengths."""
    p = K.kaze_default_params()
    p.scheme = K.KAZE_FED
    kz = K.Kaze(W, H, p)
    for _ in range(max(2, args.warmup // 4)):
        kz.run(img)
    torch.cuda.synchronize()
    steps = max(5, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        kz.run(img)
    torch.cuda.synchronize()
    val = steps / (time.perf_counter() - t0)
    per = {}
    for name in ("fed", "cond"):
        K.kaze_profile_begin(name)
        for _ in range(3):
            kz.run(img)
        n, ms = K.kaze_profile_end()
        per[name] = (n / 3, 1e3 * ms / 3)
    sched = K.kaze_schedule(p)
    cycles = [len(K.kaze_fed_schedule(sched[i]["tau"])) for i in range(1, kz.N)]
    level_us = (per["fed"][1] + per["cond"][1]) / (kz.N - 1)  # us per image / steps
    return {"images_per_s": round(val, 3), "path": "eager calls",
            "explicit_steps_per_image": int(sum(cycles)),
            "launches_per_image": int(per["fed"][0]),
            "us_per_level": round(level_us, 3),
            "speedup_vs_plain_aos_eager": round(val / plain_eager, 4),
            "speedup_vs_plain_aos_graph": round(val / plain_value, 4)}


def bench_substeps(args, K, torch, img, W, H, plain_eager):
    """m AOS sub-steps per level (each recomputing the conductivity): eager
    images/s and the time of one sub-step (event pairs around the AOS
    launches)."""
    out = {}
    for m in (2, 4):
        kz = K.Kaze(W, H, K.kaze_default_params(substeps=m))
        for _ in range(2):
            kz.run(img)
        torch.cuda.synchronize()
        steps = max(20, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(steps):
            kz.run(img)
        torch.cuda.synchronize()
        val = steps / (time.perf_counter() - t0)
        K.kaze_profile_begin(",".join(AOS_KERNELS))
        kz.run(img)
        n, ms = K.kaze_profile_end()
        out[str(m)] = {"images_per_s": round(val, 3), "path": "eager calls",
                       "us_per_substep": round(1e3 * ms / (n / 3), 3),
                       "relative_to_one_step": round(val / plain_eager, 4)}
    return out


def bench_keypoints(args, K, torch, img, W, H):
    """The extrema stage with the 3x3 and the sigma x sigma cross-level
    window (nms launch time, keypoint counts), and the refinement and edge
    test of the window's extrema (refine launch time, kept count); event
    pairs around every launch, eager calls."""
    out = {}
    for name, window in (("window_3x3", K.KAZE_WINDOW_3X3), ("window_sigma", K.KAZE_WINDOW_SIGMA)):
        p = K.kaze_default_params()
        p.extrema_window = window
        kz = K.Kaze(W, H, p)
        kz.run(img)
        torch.cuda.synchronize()
        K.kaze_profile_begin("nms")
        for _ in range(10):
            kz.extrema()
        n, ms = K.kaze_profile_end()
        out[name] = {"keypoints": int(kz.count.item()), "nms_us": round(1e3 * ms / n, 3)}
    kz.refine()
    torch.cuda.synchronize()
    K.kaze_profile_begin("refine")
    for _ in range(10):
        kz.refine()
    n, ms = K.kaze_profile_end()
    kept = int(kz.refined_keypoints()[:, 5].sum())
    out["refine"] = {"keypoints": int(kz.count.item()), "kept": kept,
                     "us_per_launch": round(1e3 * ms / n, 3), "edge_ratio": 10.0}
    kz.describe()
    torch.cuda.synchronize()
    for name in ("deriv", "describe"):
        K.kaze_profile_begin(name)
        for _ in range(10):
            kz.describe()
        n, ms = K.kaze_profile_end()
        out[name] = {"us_per_launch": round(1e3 * ms / n, 3)}
    out["describe"]["keypoints"] = int(kz.count.item())
    out["deriv"]["levels"] = kz.N
    return out


def bench_surrogate(args, K, torch, img, W, H, seed, plain_value):
    """The surrogate form on the same image: the default per-level check and
    fallback, and every level forced to the surrogate (its cost without
    checks); plus the MFMA roofline of the hidden 32 -> 32 convolution."""
    import math
    from paper_1706_06750_amd import surrogate as S
    from paper_1706_06750_amd import train_surrogate as T
    if not os.path.exists(T.DEFAULT_OUT):
        return {"skipped": "no trained weights (%s)" % os.path.relpath(T.DEFAULT_OUT, ROOT)}
    params, meta = T.load()
    w = S.Weights(params)
    out = {"weights": os.path.relpath(T.DEFAULT_OUT, ROOT),
           "trained_on": "%d images %dx%d, %d epochs" % (meta["images"], meta["size"],
                                                         meta["size"], meta["epochs"])}
    steps = max(5, args.steps // 4)
    for name, cfg in (("default", {}), ("all_surrogate", {"bound": math.inf, "probes": 0})):
        c = S.kaze_sg_default_config(**cfg)
        ss = S.SurrogateScaleSpace(W, H, w, config=c, probe_seed=seed)
        ss.img.copy_(img)
        for _ in range(max(2, args.warmup // 4)):
            ss.run()
        torch.cuda.synchronize()
        K.kaze_profile_begin("aos_reduce")
        t0 = time.perf_counter()
        for _ in range(steps):
            ss.run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs, ms = K.kaze_profile_end()
        acc = ss.accepted()
        val = steps / el
        out[name] = {"bound": c.bound, "probes": c.probes, "images_per_s": round(val, 3),
                     "us_per_level": round(1e3 * ms / (runs * (ss.N - 1)), 3),
                     "levels_accepted": int(sum(acc)),
                     "accepted": [int(a) for a in acc],
                     "probe_err": [float("%.3e" % e) for e in ss.err.cpu().tolist()],
                     "speedup_vs_plain": round(val / plain_value, 4)}
        if name == "all_surrogate":
            # eager run with events around every hidden-layer launch
            K.kaze_profile_begin("sg_conv")
            for _ in range(2):
                ss.run(eager=True)
            n, cms = K.kaze_profile_end()
            us = 1e3 * cms / n
            flop = CONV_FLOP_PER_PX * W * H
            tf = flop / (us * 1e-6) / 1e12
            out["conv_roofline"] = {"kernel": "conv2_kernel<32, 2> (layers 3 and 4 fused)",
                                    "bound": "mfma", "achieved": round(tf, 1),
                                    "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(tf / BF16_PEAK_TFLOPS, 4),
                                    "flop_per_launch": flop, "us_per_launch": round(us, 3)}
        ss.close()
    return out


IMAGE_WORKER_SRC = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
from synthetic import kaze_image
for (W, H, seed, path) in %r:
    np.save(path, kaze_image(W, H, seed))
"""


def parallel_images(cases, workers=16):
    """Inputs of a workload generated by child processes (the generator is
    pure NumPy; the children never touch the GPU), loaded back in order."""
    import tempfile

    import numpy as np
    tmp = tempfile.mkdtemp(prefix="kaze_inputs_")
    jobs = [(W, H, seed, os.path.join(tmp, "img%03d.npy" % j)) for j, (W, H, seed) in enumerate(cases)]
    P = max(1, min(workers, len(os.sched_getaffinity(0)), len(jobs)))
    procs = [subprocess.Popen([sys.executable, "-c", IMAGE_WORKER_SRC % (ROOT, jobs[w::P])],
                              stderr=subprocess.PIPE, text=True) for w in range(P)]
    for pr in procs:
        _, err = pr.communicate(timeout=600)
        if pr.returncode != 0:
            raise RuntimeError("input generation failed: " + err[-2000:])
    out = []
    for _, _, _, path in jobs:
        out.append(np.load(path))
        os.unlink(path)
    os.rmdir(tmp)
    return out


def measure_plan(args, K, torch, kb, sizes, traffic_key, steps):
    """Times both launch forms of a created plan over `steps` runs and returns
    the faster with its level-segment roofline."""
    saved = args.steps, args.warmup
    args.steps, args.warmup = steps, max(2, min(args.warmup, steps // 2))
    try:
        elapsed, level_us, form, forms = timed_plan(args, K, torch, kb, len(sizes))
    finally:
        args.steps, args.warmup = saved
    px = sum(W * H for W, H in sizes)
    dl = det_levels_of(kb, form)
    roof = level_roofline(level_us, px,
                          traffic_from_profile(traffic_key, tile_label(K, kb.shape), dl)
                          if traffic_key else None,
                          det_levels=dl)
    roof["timed_in"] = "the timed region (event pair around each run's AOS segment)"
    return {"images_per_s": round(len(sizes) * steps / elapsed, 3),
            "megapixels_per_s": round(px * steps / elapsed / 1e6, 1),
            "ms_per_run": round(1e3 * elapsed / steps, 4), "steps": steps,
            "path": "plain AOS, batched, %s" % ("eager launches" if form == "eager"
                                                else "graph replay"),
            "aos_tile": tile_label(K, kb.shape), "autotune_ms_per_shape": kb.tune_ms,
            "plan_launch_forms": forms, "roofline": roof}


def batch_config(workload, sizes, N):
    px = sum(W * H for W, H in sizes)
    return {"workload": workload, "images": len(sizes), "pixels": px,
            "sizes": "W in [%d,%d], H in [%d,%d]" % (min(w for w, _ in sizes),
                                                     max(w for w, _ in sizes),
                                                     min(h for _, h in sizes),
                                                     max(h for _, h in sizes)),
            "levels": N}


def bench_batch(args, K, torch, kaze_image, cases):
    """--workload of several images: the plain batched path is the record."""
    sizes = [(W, H) for W, H, _ in cases]
    kb = K.KazeBatch(sizes, shape="auto", capacity=1 << 12)
    imgs = parallel_images(cases) if len(cases) > 8 else [kaze_image(*c) for c in cases]
    for x, im in zip(kb.inputs, imgs):
        x.copy_(torch.from_numpy(im))
    m = measure_plan(args, K, torch, kb, sizes, args.workload.replace("kaze_", ""), args.steps)
    config = batch_config(args.workload, sizes, kb.N)
    config.update(path=m["path"], aos_tile=m["aos_tile"],
                  autotune_ms_per_shape=m["autotune_ms_per_shape"])
    extra = {"megapixels_per_s": m["megapixels_per_s"], "plan_launch_forms": m["plan_launch_forms"]}
    kb.close()
    del kb
    torch.cuda.empty_cache()
    if not args.no_surrogate and args.workload == "kaze_4k32_720p32":
        extra["surrogate"] = bench_surrogate_batch(args, K, torch, cases, imgs, m["images_per_s"])
    return record(args, m["images_per_s"], m["ms_per_run"], config, m["roofline"], extra)


def bench_batches(args, K, torch, kaze_image):
    """Batches beside the single-image record: the 64-image uneven batch and
    eight 1920x1200 images (plain path, autotuned tile, each with its own
    level-segment roofline), and the 4K + 720p workload through the plain
    batched path and the batched surrogate."""
    from synthetic import WORKLOADS
    out = {}
    for name, steps in (("kaze_batch64_uneven", 20), ("kaze_8x1920x1200", 20)):
        cases = WORKLOADS[name]()
        sizes = [(W, H) for W, H, _ in cases]
        imgs = parallel_images(cases)
        kb = K.KazeBatch(sizes, shape="auto", capacity=1 << 12)
        for x, im in zip(kb.inputs, imgs):
            x.copy_(torch.from_numpy(im))
        m = measure_plan(args, K, torch, kb, sizes, name.replace("kaze_", ""), steps)
        m["config"] = batch_config(name, sizes, kb.N)
        kb.close()
        del kb, imgs
        torch.cuda.empty_cache()
        out[name] = m
        progress("%s: %.1f images/s, %.1f%% of HBM peak per level" %
                 (name, m["images_per_s"], 100 * m["roofline"]["frac"]))
    if not args.no_surrogate:
        cases = WORKLOADS["kaze_4k32_720p32"]()
        sizes = [(W, H) for W, H, _ in cases]
        imgs = parallel_images(cases)
        kb = K.KazeBatch(sizes, shape="auto", capacity=1 << 12)
        for x, im in zip(kb.inputs, imgs):
            x.copy_(torch.from_numpy(im))
        m = measure_plan(args, K, torch, kb, sizes, "4k32_720p32", 5)
        m["config"] = batch_config("kaze_4k32_720p32", sizes, kb.N)
        progress("kaze_4k32_720p32 plain batched: %.1f images/s" % m["images_per_s"])
        m["surrogate"] = bench_surrogate_batch(args, K, torch, cases, imgs, m["images_per_s"],
                                               plain=kb)
        kb.close()
        del kb, imgs
        torch.cuda.empty_cache()
        out["kaze_4k32_720p32"] = m
    return out


def bench_surrogate_batch(args, K, torch, cases, imgs, plain_value, plain=None):
    """The batched surrogate form (one plan for every image; per image and
    level the probe check, the network where accepted, AOS where rejected)
    on the workload: default check and every level forced to the network,
    images/s against the plain batched path, the levels accepted and every
    image's largest difference from the plain batched levels (when `plain`,
    a plain plan that has run on the same inputs, is given).  Errors against
    the FP64 oracle on this workload are measured by the GPU tests."""
    import math

    import numpy as np
    from paper_1706_06750_amd import surrogate as S
    from paper_1706_06750_amd import train_surrogate as T
    if not os.path.exists(T.DEFAULT_OUT):
        return {"skipped": "no trained weights"}
    params, _ = T.load()
    w = S.Weights(params)
    sizes = [(W, H) for W, H, _ in cases]
    out = {"plan": "kaze_sg_batch_create: every phase one launch over the %d images" % len(sizes)}
    for name, cfg in (("default", {}), ("all_surrogate", {"bound": math.inf, "probes": 0})):
        c = S.kaze_sg_default_config(**cfg)
        sb = S.SurrogateBatch(sizes, w, config=c, probe_seed=cases[0][2], capacity=1 << 12)
        for x, im in zip(sb.inputs, imgs):
            x.copy_(torch.from_numpy(im))
        sb.run()
        torch.cuda.synchronize()
        steps = 3
        K.kaze_profile_begin("aos_reduce")
        t0 = time.perf_counter()
        for _ in range(steps):
            sb.run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs, ms = K.kaze_profile_end()
        acc = sb.accepted()
        val = len(sizes) * steps / el
        r = {"bound": c.bound, "probes": c.probes, "images_per_s": round(val, 3),
             "ms_per_run": round(1e3 * el / steps, 3),
             "us_per_level": round(1e3 * ms / (max(runs, 1) * (sb.N - 1)), 3),
             "levels_accepted": int(acc.sum()), "level_decisions": int(acc[:, 1:].size),
             "accepted_levels_per_image": acc.sum(axis=1).tolist(),
             "speedup_vs_plain_batched": round(val / plain_value, 4)}
        if name == "default":
            pe = sb.err.cpu().numpy()[:, 1:]
            r["probe_err_range"] = [float("%.3e" % pe.min()), float("%.3e" % pe.max())]
            if plain is not None:
                d = [float((sb.levels[j] - plain.levels[j]).abs().max().item())
                     for j in range(len(sizes))]
                r["max_abs_vs_plain_batched_per_image"] = [float("%.3e" % v) for v in d]
                r["keypoints_equal_plain_batched"] = int(sum(
                    int(np.array_equal(sb.keypoints(j), plain.keypoints(j)))
                    for j in range(len(sizes))))
        out[name] = r
        sb.close()
        del sb
        torch.cuda.empty_cache()
        progress("surrogate batch (%s): %.1f images/s" % (name, r["images_per_s"]))
    return out


if __name__ == "__main__":
    main()
