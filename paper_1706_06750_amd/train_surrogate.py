"""Train the AOS-step surrogate on the GPU.

Training pairs come from the plain method on the fly: for every synthetic
image the library builds the scale space, and each step i -> i+1 gives one
pair (L_{i-1}, g(L_{i-1}), tau_i) -> L_i.  Each pair's loss is weighted by
1 / tau_i: a step moves a level by an amount that grows with tau (about 12x
from the first to the last level), and unweighted the large steps would
decide the whole fit.  The forward pass, the backward pass and Adam run in
libkaze's MFMA kernels; this module only schedules them and moves tensors.

    python -m paper_1706_06750_amd.train_surrogate [--images 2000] [--size 512]
        [--epochs 3] [--batch 16] [--lr 1e-3] [--levels 1-3] [--out weights/surrogate_512.npz]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synthetic import kaze_image, surrogate_params  # noqa: E402

DEFAULT_OUT = os.path.join(PKG_DIR, "weights", "surrogate_512.npz")


def _gen(args):
    W, seed = args
    return kaze_image(W, W, seed)


def make_images(n, size, seed0, workers):
    """n seeded size x size images (seeds seed0 + j) as one float32 array."""
    jobs = [(size, seed0 + j) for j in range(n)]
    if workers <= 1:
        return np.stack([_gen(j) for j in jobs])
    with ProcessPoolExecutor(workers) as ex:
        return np.stack(list(ex.map(_gen, jobs, chunksize=8)))


class PairSource:
    """Level pairs of a chunk of images from the plain GPU path (the steps
    into the levels in `levels`, default every level 1..N-1)."""

    def __init__(self, K, size, chunk, levels=None):
        import torch
        self.K, self.size, self.chunk = K, size, chunk
        self.kb = K.KazeBatch([(size, size)] * chunk, shape=0, with_detector=False)
        self.N = self.kb.N
        self.levels = list(levels) if levels else list(range(1, self.N))
        sched = K.kaze_schedule(self.kb.p)
        self.tau = torch.tensor([s["tau"] for s in sched], dtype=torch.float32, device="cuda")
        n = chunk * len(self.levels)
        self.L = torch.empty((n, size, size), device="cuda")
        self.g = torch.empty_like(self.L)
        self.Ln = torch.empty_like(self.L)
        self.t = torch.empty(n, device="cuda")

    def fill(self, images):
        """images: [chunk][size][size] device tensor -> pairs in L, g, Ln, t."""
        K, s = self.K, self.size
        for j in range(self.chunk):
            self.kb.inputs[j].copy_(images[j])
        self.kb.run()
        r = 0
        for j in range(self.chunk):
            lev = self.kb.levels[j]
            k = float(self.kb.k[j].item())
            for i in self.levels:
                self.L[r].copy_(lev[i - 1])
                self.Ln[r].copy_(lev[i])
                K.kaze_conductivity(lev[i - 1], s, s, self.kb.p, k, self.g[r])
                self.t[r] = self.tau[i]
                r += 1
        return r


def evaluate(K, S, w, size=512, images=16, image_seed=410000, workers=None, chunk=16):
    """Per-level error of the network on held-out level pairs (images not
    used in training): RMS and max |f - (L_i - L_{i-1})|, next to the same
    figures for taking no step at all (f = 0)."""
    import torch
    host = make_images(images, size, image_seed, workers or 1)
    imgs = torch.from_numpy(host).cuda()
    src = PairSource(K, size, chunk)
    N = src.N
    plan = S.Plan(chunk * (N - 1), size, size, training=False)
    sq = np.zeros(N)
    mx = np.zeros(N)
    sq0 = np.zeros(N)
    mx0 = np.zeros(N)
    cnt = 0
    for c in range(images // chunk):
        src.fill(imgs[c * chunk:(c + 1) * chunk])
        f = plan.forward(w, src.L, src.g, src.t, add_input=False)
        r = (f - (src.Ln - src.L)).reshape(chunk, N - 1, -1)
        d = (src.Ln - src.L).reshape(chunk, N - 1, -1)
        sq[1:] += (r.double() ** 2).mean(dim=2).sum(dim=0).cpu().numpy()
        mx[1:] = np.maximum(mx[1:], r.abs().amax(dim=(0, 2)).cpu().numpy())
        sq0[1:] += (d.double() ** 2).mean(dim=2).sum(dim=0).cpu().numpy()
        mx0[1:] = np.maximum(mx0[1:], d.abs().amax(dim=(0, 2)).cpu().numpy())
        cnt += chunk
    return {"rms": np.sqrt(sq / cnt).tolist(), "max": mx.tolist(),
            "rms_no_step": np.sqrt(sq0 / cnt).tolist(), "max_no_step": mx0.tolist(),
            "images": images, "image_seed": image_seed}


def train(images=2000, size=512, epochs=3, batch=16, lr=1e-3, lr_min=1e-5, chunk=16, seed=0,
          image_seed=400000, workers=None, log_every=100, out=DEFAULT_OUT, verbose=True,
          levels=None):
    import torch
    from . import kaze as K
    from . import surrogate as S

    workers = workers or min(16, os.cpu_count() or 1)
    t0 = time.time()
    host = make_images(images, size, image_seed, workers)
    imgs = torch.from_numpy(host).cuda()
    del host
    t_gen = time.time() - t0
    src = PairSource(K, size, chunk, levels)
    w = S.Weights(surrogate_params(seed))
    plan = S.Plan(batch, size, size, training=True)
    rng = np.random.default_rng(seed + 1)
    pairs_per_chunk = chunk * len(src.levels)
    steps_per_chunk = pairs_per_chunk // batch
    n_chunks = images // chunk
    total = epochs * n_chunks * steps_per_chunk
    history = []
    step = 0
    torch.cuda.synchronize()
    t1 = time.time()
    for ep in range(epochs):
        order = rng.permutation(n_chunks)
        for c in order:
            src.fill(imgs[c * chunk:(c + 1) * chunk])
            perm = torch.from_numpy(rng.permutation(pairs_per_chunk)).cuda()
            for b in range(steps_per_chunk):
                idx = perm[b * batch:(b + 1) * batch]
                L = src.L.index_select(0, idx)
                g = src.g.index_select(0, idx)
                Ln = src.Ln.index_select(0, idx)
                tau = src.t.index_select(0, idx)
                loss = plan.gradients(w, L, g, tau, Ln, weight=1.0 / tau)
                cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(1, total)))
                w.adam(lr=cur)
                step += 1
                if step % log_every == 0 or step == total:
                    lv = float(loss.item())
                    history.append((step, lv))
                    if verbose:
                        print("step %d/%d epoch %d loss %.4e lr %.2e %.1fs" %
                              (step, total, ep, lv, cur, time.time() - t1), flush=True)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    params = w.params.cpu().numpy()
    held = evaluate(K, S, w, size, workers=workers)
    if verbose:
        print("held-out per-level RMS  %s" % " ".join("%.1e" % v for v in held["rms"][1:]))
        print("held-out per-level max  %s" % " ".join("%.1e" % v for v in held["max"][1:]))
        print("no step: per-level max  %s" % " ".join("%.1e" % v for v in held["max_no_step"][1:]))
    meta = {"images": images, "size": size, "epochs": epochs, "batch": batch, "lr": lr,
            "lr_min": lr_min, "chunk": chunk, "init_seed": seed, "image_seed": image_seed,
            "steps": step, "pairs_per_epoch": n_chunks * pairs_per_chunk, "levels": src.levels,
            "image_generation_s": round(t_gen, 2), "train_s": round(t_train, 2),
            "held_out": held, "loss_history": history}
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        np.savez(out, params=params, meta=json.dumps(meta))
    return params, meta


def load(path=DEFAULT_OUT):
    """(params float32, meta dict) of a saved surrogate."""
    d = np.load(path, allow_pickle=False)
    return d["params"].astype(np.float32), json.loads(str(d["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--images", type=int, default=2000)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=None)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--levels", default=None,
                    help="train on the steps into levels lo-hi only (e.g. 1-3); default all")
    a = ap.parse_args()
    levels = None
    if a.levels:
        lo, hi = (int(v) for v in a.levels.split("-"))
        levels = range(lo, hi + 1)
    _, meta = train(a.images, a.size, a.epochs, a.batch, a.lr, chunk=a.chunk, seed=a.seed,
                    workers=a.workers, out=a.out, levels=levels)
    print(json.dumps({k: v for k, v in meta.items() if k != "loss_history"}))


if __name__ == "__main__":
    main()
