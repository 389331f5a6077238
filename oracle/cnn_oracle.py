"""FP64 CPU oracle of the learned surrogate for one AOS step.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke entry
point and the CPU-baseline leg of the benchmark may import this module.  It
shares no code with the GPU library.

The paper builds the scale space with semi-implicit steps (Sec. II-A, Eq. 4)
and mentions learned diffusion models only as related work (trainable
nonlinear reaction diffusion, Sec. V).  The surrogate below is therefore not
defined by the paper; this module is the definition the GPU kernels are
checked against:

* input planes X0 = (L, g, tau / TAU_REF) of one level step, where L is the
  previous level, g its conductivity and tau the step's time increment;
* six 3x3 convolutions (cross-correlation, zero padding of one pixel) with
  channel counts 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, bias per output
  channel, ReLU after layers 1..5, nothing after layer 6;
* the network output f is OUT_SCALE times the output of layer 6 and is the
  residual of the step: L_next ~ L + f.  One step moves a level by about
  1e-3 (RMS) while the hidden activations are of order one; the fixed
  power-of-two scale lets layer 6 work at order-one values;
* loss: mean over every pixel of every sample of w_s (f - (L_next - L))^2,
  with a weight w_s per sample (1 unless given; training uses 1 / tau so
  that the small steps of the first levels count as much as the large ones
  of the last);
* Adam (Kingma and Ba 2015) with bias correction on the flat FP32 parameter
  vector.

Parameters are one flat vector: for each layer the weights [co][ci][3][3]
followed by the biases [co] (38,177 values in all).

``quantized=True`` selects the storage precisions of the GPU kernels, stated
here as part of the definition and evaluated otherwise in float64:
layer 1 is exact (the GPU evaluates it to ~2^-16 relative error with a
three-term BF16 split of inputs and weights); weights of layers 2..6 are
rounded to BF16; the outputs of layers 1..5 are rounded to BF16 after the
ReLU; f is not rounded.  In the backward pass the gradient entering each
layer (dZ) is rounded to BF16 and the rounded weights are used for the
transposed convolutions (straight-through estimate for the weight rounding).
BF16 rounding is round-to-nearest-even of the float32 value.
"""
from __future__ import annotations

import numpy as np

from . import kaze_oracle as K

__all__ = [
    "TAU_REF", "OUT_SCALE", "CHANNELS", "param_shapes", "param_count", "unflatten",
    "flatten", "bf16_round", "conv3x3", "conv3x3_input_grad",
    "conv3x3_weight_grad", "input_planes", "forward", "backward",
    "loss_and_grad", "adam_step", "surrogate_step", "surrogate_scale_space",
]

TAU_REF = 68.0
OUT_SCALE = 1.0 / 64.0
CHANNELS = (3, 32, 32, 32, 32, 32, 1)


def param_shapes():
    """[(weight shape, bias shape)] per layer."""
    return [((co, ci, 3, 3), (co,)) for ci, co in zip(CHANNELS[:-1], CHANNELS[1:])]


def param_count() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unflatten(theta):
    """Flat vector -> [(W, b)] (views into a float64 copy)."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (param_count(),):
        raise ValueError("expected %d parameters" % param_count())
    out, o = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value, ties to even, via float32 (returned as
    float64).  BF16 keeps the sign, the 8 exponent bits and the top 7
    mantissa bits of a float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def _pad(X):
    return np.pad(X, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3x3(X, W, b):
    """Z[n,co,y,x] = b[co] + sum_{ci,dy,dx} W[co,ci,dy+1,dx+1] X[n,ci,y+dy,x+dx],
    X taken as zero outside the image.  X: [n][ci][H][W]."""
    n, ci, H, Wd = X.shape
    Xp = _pad(X)
    Z = np.zeros((n, W.shape[0], H, Wd))
    for ty in range(3):
        for tx in range(3):
            Z += np.einsum("oc,nchw->nohw", W[:, :, ty, tx], Xp[:, :, ty:ty + H, tx:tx + Wd])
    return Z + b[None, :, None, None]


def conv3x3_input_grad(dZ, W):
    """Gradient of sum(dZ * conv3x3(X, W, b)) with respect to X: each output
    pixel p sends W[:, :, t]^T dZ[p] to input pixel p + t (if inside)."""
    n, co, H, Wd = dZ.shape
    dXp = np.zeros((n, W.shape[1], H + 2, Wd + 2))
    for ty in range(3):
        for tx in range(3):
            dXp[:, :, ty:ty + H, tx:tx + Wd] += np.einsum("oc,nohw->nchw", W[:, :, ty, tx], dZ)
    return dXp[:, :, 1:H + 1, 1:Wd + 1]


def conv3x3_weight_grad(X, dZ):
    """Gradients with respect to W and b of sum(dZ * conv3x3(X, W, b))."""
    n, ci, H, Wd = X.shape
    Xp = _pad(X)
    dW = np.zeros((dZ.shape[1], ci, 3, 3))
    for ty in range(3):
        for tx in range(3):
            dW[:, :, ty, tx] = np.einsum("nohw,nchw->oc", dZ, Xp[:, :, ty:ty + H, tx:tx + Wd])
    return dW, dZ.sum(axis=(0, 2, 3))


def input_planes(L, g, tau):
    """X0 for a batch: L, g [n][H][W], tau [n] -> [n][3][H][W]."""
    L = np.asarray(L, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if L.ndim == 2:
        L, g = L[None], g[None]
    tau = np.broadcast_to(np.asarray(tau, dtype=np.float64).reshape(-1), (L.shape[0],))
    T = np.broadcast_to((tau / TAU_REF)[:, None, None], L.shape)
    return np.stack([L, g, T], axis=1)


def forward(theta, L, g, tau, quantized=False):
    """Network output f [n][H][W] and the per-layer inputs (for ``backward``)."""
    layers = unflatten(theta)
    X = input_planes(L, g, tau)
    acts = [X]
    for li, (W, b) in enumerate(layers):
        Wl = bf16_round(W) if (quantized and li > 0) else W
        Z = conv3x3(X, Wl, b)
        if li == len(layers) - 1:
            return OUT_SCALE * Z[:, 0], acts
        X = np.maximum(Z, 0.0)
        if quantized:
            X = bf16_round(X)
        acts.append(X)
    raise AssertionError("unreachable")


def backward(theta, acts, dF, quantized=False):
    """Gradient of sum(dF * f) with respect to the flat parameter vector."""
    layers = unflatten(theta)
    dZ = OUT_SCALE * np.asarray(dF, dtype=np.float64)[:, None]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        Wl = bf16_round(W) if (quantized and li > 0) else W
        if quantized:
            dZ = bf16_round(dZ)
        grads[li] = conv3x3_weight_grad(acts[li], dZ)
        if li == 0:
            break
        dX = conv3x3_input_grad(dZ, Wl)
        dZ = dX * (acts[li] > 0)
    return flatten(grads)


def loss_and_grad(theta, L, g, tau, L_next, quantized=False, weights=None):
    """(loss, grad, f) for the weighted residual MSE of one batch of level
    steps (weights: one per sample, default 1)."""
    L = np.asarray(L, dtype=np.float64)
    L_next = np.asarray(L_next, dtype=np.float64)
    if L.ndim == 2:
        L, L_next, g = L[None], L_next[None], np.asarray(g)[None]
    f, acts = forward(theta, L, g, tau, quantized)
    r = f - (L_next - L)
    w = np.ones(L.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64).reshape(-1)
    wr = w[:, None, None] * r
    loss = float(np.sum(wr * r) / r.size)
    dF = 2.0 * wr / r.size
    return loss, backward(theta, acts, dF, quantized), f


def adam_step(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def surrogate_step(theta, L, g, tau, quantized=False):
    """L_next ~ L + f(L, g, tau) for one image [H][W]."""
    f, _ = forward(theta, L, g, tau, quantized)
    return np.asarray(L, dtype=np.float64) + f[0]


def surrogate_scale_space(img, theta, accept, quantized=False, sigma0=1.6, octaves=4,
                          sublevels=4, sigma_cond=1.0, k=None):
    """Scale space whose step into level i is the surrogate where ``accept[i]``
    is true and the exact AOS step (Eq. 4) otherwise.  The base level, the
    contrast factor and every conductivity follow the plain method; g is
    always taken from the level actually produced.  Returns (levels, k)."""
    f = np.asarray(img, dtype=np.float64)
    sched = K.level_schedule(sigma0, octaves, sublevels)
    L0 = K.gaussian_smooth(f, sigma0)
    if k is None:
        k = K.contrast_factor(L0, sigma_cond)
    levels = [L0]
    for i in range(1, len(sched)):
        g = K.conductivity_g2(levels[-1], k, sigma_cond)
        tau = sched[i]["t"] - sched[i - 1]["t"]
        if accept[i]:
            levels.append(surrogate_step(theta, levels[-1], g, tau, quantized))
        else:
            levels.append(K.aos_step(levels[-1], g, tau))
    return np.stack(levels), float(k)
