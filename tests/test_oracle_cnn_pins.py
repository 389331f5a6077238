"""Pins of the FP64 surrogate oracle against facts that do not come from it:
brute-force loops, a library correlation, closed forms of special networks,
central finite differences, Adam's closed-form first steps and the BF16
conversion of a library."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_oracle as C
from synthetic import kaze_image, surrogate_params


def brute_conv(X, W, b):
    """Pure-Python loops over every index (tiny inputs only)."""
    n, ci, H, Wd = X.shape
    co = W.shape[0]
    Z = np.zeros((n, co, H, Wd))
    for a in range(n):
        for o in range(co):
            for y in range(H):
                for x in range(Wd):
                    s = b[o]
                    for c in range(ci):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                yy, xx = y + dy, x + dx
                                if 0 <= yy < H and 0 <= xx < Wd:
                                    s += W[o, c, dy + 1, dx + 1] * X[a, c, yy, xx]
                    Z[a, o, y, x] = s
    return Z


def test_param_count_matches_architecture():
    # 3->32, four 32->32, 32->1, 3x3 kernels with biases
    assert C.param_count() == (3 * 32 * 9 + 32) + 4 * (32 * 32 * 9 + 32) + (32 * 9 + 1) == 38177
    th = surrogate_params(0)
    assert th.shape == (38177,) and th.dtype == np.float32
    assert np.array_equal(C.flatten(C.unflatten(th)), th.astype(np.float64))


def test_conv_matches_brute_force_and_library():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2, 3, 7, 6))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    Z = C.conv3x3(X, W, b)
    assert np.allclose(Z, brute_conv(X, W, b), rtol=0, atol=1e-12)
    # library cross-correlation with zero fill, summed over input channels
    for a in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(X[a, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(Z[a, o], ref, rtol=0, atol=1e-12)


def test_transposed_conv_is_the_adjoint():
    """<conv(X) - b, Y> = <X, conv^T(Y)> and <conv(X) - b, Y> = <W, dW(X, Y)>."""
    rng = np.random.default_rng(6)
    X = rng.normal(size=(2, 5, 6, 9))
    Y = rng.normal(size=(2, 4, 6, 9))
    W = rng.normal(size=(4, 5, 3, 3))
    b = np.zeros(4)
    lhs = np.sum(C.conv3x3(X, W, b) * Y)
    assert np.isclose(lhs, np.sum(X * C.conv3x3_input_grad(Y, W)), rtol=1e-12)
    dW, db = C.conv3x3_weight_grad(X, Y)
    assert np.isclose(lhs, np.sum(W * dW), rtol=1e-12)
    assert np.allclose(db, Y.sum(axis=(0, 2, 3)))


def test_zero_last_layer_is_the_identity_step():
    th = surrogate_params(1).astype(np.float64)
    layers = C.unflatten(th)
    layers[-1][0][...] = 0.0
    layers[-1][1][...] = 0.0
    th0 = C.flatten(layers)
    L = kaze_image(24, 17, 3).astype(np.float64)
    g = np.full_like(L, 0.7)
    assert np.array_equal(C.surrogate_step(th0, L, g, 2.0), L)


def identity_net(a, c_tau, bias6):
    """Layers 1..5 copy the three input planes through the centre tap (inputs
    are positive, so the ReLUs pass them); layer 6 weights them."""
    layers = []
    for ci, co in zip(C.CHANNELS[:-2], C.CHANNELS[1:-1]):
        W = np.zeros((co, ci, 3, 3))
        for k in range(3):
            W[k, k, 1, 1] = 1.0
        layers.append((W, np.zeros(co)))
    W6 = np.zeros((1, 32, 3, 3))
    W6[0, 0, 1, 1], W6[0, 1, 1, 1], W6[0, 2, 1, 1] = a
    layers.append((W6, np.array([bias6])))
    return C.flatten(layers)


def test_identity_network_closed_form():
    a = (0.5, -0.25, 2.0)
    th = identity_net(a, None, 0.125)
    L = kaze_image(20, 14, 4).astype(np.float64) + 0.1
    g = np.linspace(0.2, 1.0, L.size).reshape(L.shape)
    tau = 17.0
    f, _ = C.forward(th, L, g, tau)
    ref = C.OUT_SCALE * (a[0] * L + a[1] * g + a[2] * tau / C.TAU_REF + 0.125)
    assert np.allclose(f[0], ref, rtol=0, atol=1e-14)
    # every intermediate value is exactly representable: the BF16 storage
    # rounding changes nothing when weights and planes are BF16 numbers
    Lq = C.bf16_round(L)
    gq = C.bf16_round(g)
    tq = 0.5 * C.TAU_REF   # tau / TAU_REF = 0.5
    fq, _ = C.forward(th, Lq, gq, tq, quantized=True)
    fx, _ = C.forward(th, Lq, gq, tq, quantized=False)
    assert np.array_equal(fq, fx)


def test_translation_equivariance_away_from_borders():
    th = surrogate_params(2).astype(np.float64)
    L = kaze_image(40, 30, 6).astype(np.float64)
    g = np.full_like(L, 0.5)
    f, _ = C.forward(th, L, g, 3.0)
    Ls = np.roll(L, (2, 3), axis=(0, 1))
    fs, _ = C.forward(th, Ls, g, 3.0)
    # receptive field 13x13: pixels 6 from every border (of both) agree
    assert np.allclose(fs[0, 2 + 6:-6, 3 + 6:-6], f[0, 6:-6 - 2, 6:-6 - 3], atol=1e-13)


@pytest.mark.parametrize("quantized", [False])
def test_gradient_by_central_differences(quantized):
    rng = np.random.default_rng(7)
    th = surrogate_params(3).astype(np.float64)
    th[C.param_count() - 1] = 0.01
    n, H, W = 2, 9, 9
    L = rng.uniform(0, 1, size=(n, H, W))
    g = rng.uniform(0.1, 1, size=(n, H, W))
    Ln = L + 0.05 * rng.normal(size=(n, H, W))
    tau = np.array([1.5, 30.0])
    loss, grad, _ = C.loss_and_grad(th, L, g, tau, Ln)
    # probe parameters of every layer (weights and biases)
    idx, o = [], 0
    for ws, bs in C.param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        idx += list(o + rng.choice(nw, 6, replace=False)) + [o + nw + int(rng.integers(nb))]
        o += nw + nb
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (C.loss_and_grad(tp, L, g, tau, Ln)[0] - C.loss_and_grad(tm, L, g, tau, Ln)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * abs(grad[i]) + 1e-11, (i, fd, grad[i])


def test_input_gradient_by_central_differences():
    """The transposed convolutions (dX) of the chain, probed through L."""
    rng = np.random.default_rng(8)
    th = surrogate_params(4).astype(np.float64)
    L = rng.uniform(0, 1, size=(1, 8, 10))
    g = rng.uniform(0.1, 1, size=(1, 8, 10))
    layers = C.unflatten(th)
    w = rng.normal(size=(1, 8, 10))

    def obj(Lx):
        f, _ = C.forward(th, Lx, g, 2.0)
        return float(np.sum(w * f))

    f, acts = C.forward(th, L, g, 2.0)
    # dObj/dX0 by chaining the oracle's transposed convolutions by hand
    dZ = C.OUT_SCALE * w[:, None]
    for li in range(5, 0, -1):
        dX = C.conv3x3_input_grad(dZ, layers[li][0])
        dZ = dX * (acts[li] > 0)
    dX0 = C.conv3x3_input_grad(dZ, layers[0][0])[:, 0]
    h = 1e-6
    for (y, x) in [(0, 0), (3, 4), (7, 9), (5, 0)]:
        Lp, Lm = L.copy(), L.copy()
        Lp[0, y, x] += h
        Lm[0, y, x] -= h
        fd = (obj(Lp) - obj(Lm)) / (2 * h)
        assert abs(fd - dX0[0, y, x]) <= 1e-6 * abs(fd) + 1e-10


def test_quantized_backward_matches_unquantized_when_exact():
    """With BF16 numbers everywhere (identity network), the storage rounding of
    the quantized backward changes nothing."""
    th = identity_net((0.5, -0.25, 2.0), None, 0.0)
    # values on a 1/16 grid and 64 pixels: f, the residual r and dF = 2 r / 64
    # are all short binary fractions
    k = np.arange(64).reshape(1, 8, 8)
    L = 1.0 / 16 + (k % 13) / 16.0
    g = 2.0 / 16 + (k % 11) / 16.0
    Ln = L + 0.0625
    l1, g1, _ = C.loss_and_grad(th, L, g, 0.5 * C.TAU_REF, Ln, quantized=False)
    l2, g2, _ = C.loss_and_grad(th, L, g, 0.5 * C.TAU_REF, Ln, quantized=True)
    assert l1 == l2
    # dF = 2 r / n is a power-of-two multiple of r, and r is exact here
    assert np.allclose(g1, g2, rtol=0, atol=0)


def test_bf16_round_ties_and_library():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8 + 2 ** -20), 0.0, -0.0,
                  3.0e38, 1e-40, 65536.0 + 128.0, 65536.0 + 384.0])
    r = C.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie -> even mantissa
    assert r[2] == 1 + 2 ** -6               # tie -> even mantissa (upwards)
    assert r[3] == -(1 + 2 ** -7)            # above the tie -> away
    assert r[8] == 65536.0 and r[9] == 65536.0 + 512.0
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    x = np.concatenate([v, rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(x), ref)


def test_adam_closed_form_first_steps():
    g1 = np.array([0.5, -2.0, 1e-3, 0.0])
    g2 = np.array([-0.5, -1.0, 3e-3, 0.0])
    th0 = np.array([1.0, 2.0, 3.0, 4.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    th1, m, v = C.adam_step(th0, g1, np.zeros(4), np.zeros(4), 1, lr, b1, b2, eps)
    # step 1: mhat = g, vhat = g^2  ->  update -lr g/(|g|+eps)
    assert np.allclose(th1, th0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    th2, _, _ = C.adam_step(th1, g2, m, v, 2, lr, b1, b2, eps)
    mhat = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vhat = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(th2, th1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=0, atol=1e-15)


def test_loss_gradient_descends():
    """A small step against the gradient lowers the loss (FP64, no rounding)."""
    rng = np.random.default_rng(10)
    th = surrogate_params(5).astype(np.float64)
    L = rng.uniform(0, 1, size=(2, 10, 12))
    g = rng.uniform(0.1, 1, size=(2, 10, 12))
    Ln = L + 0.05
    loss, grad, _ = C.loss_and_grad(th, L, g, [1.0, 5.0], Ln)
    loss2, _, _ = C.loss_and_grad(th - 1e-3 * grad / np.linalg.norm(grad), L, g, [1.0, 5.0], Ln)
    assert loss2 < loss


def test_quantized_rounding_points_closed_form():
    """Identity network with non-BF16 weights and planes: the quantized forward
    rounds the layer-6 weights and the stored activations (layer 1 is exact),
    and the quantized backward rounds dZ before the weight gradient."""
    a = (0.5 + 2 ** -12, -0.25 - 3 * 2 ** -14, 2.0)
    th = identity_net(a, None, 0.0)
    rng = np.random.default_rng(11)
    L = rng.uniform(0.2, 0.9, size=(1, 6, 8))
    g = rng.uniform(0.2, 0.9, size=(1, 6, 8))
    tau = 11.0
    fq, acts = C.forward(th, L, g, tau, quantized=True)
    q = C.bf16_round
    ref = C.OUT_SCALE * (q(a[0]) * q(L) + q(a[1]) * q(g) + q(a[2]) * q(tau / C.TAU_REF))[0]
    assert np.allclose(fq[0], ref, rtol=0, atol=1e-15)
    # weight gradient of the centre tap of layer 6, channel 0 (L's copy)
    dF = rng.normal(size=(1, 6, 8)) * 1e-3
    grad = C.backward(th, acts, dF, quantized=True)
    W6 = C.unflatten(grad)[-1][0]
    assert np.isclose(W6[0, 0, 1, 1], np.sum(q(C.OUT_SCALE * dF) * q(L)), rtol=1e-13)
    grad_x = C.backward(th, acts, dF, quantized=False)
    assert not np.isclose(C.unflatten(grad_x)[-1][0][0, 0, 1, 1], W6[0, 0, 1, 1], rtol=1e-9)


def test_surrogate_scale_space_reduces_to_the_plain_method():
    """With every level rejected the chain is the plain oracle; with a zero
    last layer every accepted step leaves the level unchanged."""
    from oracle import kaze_oracle as K
    img = kaze_image(32, 24, 12).astype(np.float64)
    lev, k = K.build_scale_space(img)
    th = surrogate_params(6).astype(np.float64)
    lev2, k2 = C.surrogate_scale_space(img, th, [False] * 16)
    assert k2 == k and np.array_equal(lev2, lev)
    layers = C.unflatten(th)
    layers[-1][0][...] = 0.0
    lev3, _ = C.surrogate_scale_space(img, C.flatten(layers), [False] * 8 + [True] * 8)
    assert np.array_equal(lev3[8:], np.broadcast_to(lev[7], (8,) + lev[7].shape))


def test_weighted_loss_is_the_weighted_sum_of_per_sample_losses():
    rng = np.random.default_rng(13)
    th = surrogate_params(8).astype(np.float64)
    L = rng.uniform(0, 1, size=(3, 7, 9))
    g = rng.uniform(0.1, 1, size=(3, 7, 9))
    Ln = L + 0.01 * rng.normal(size=L.shape)
    tau = np.array([0.5, 3.0, 40.0])
    w = np.array([2.0, 0.25, 1.0 / 40.0])
    loss, grad, _ = C.loss_and_grad(th, L, g, tau, Ln, weights=w)
    parts = [C.loss_and_grad(th, L[j], g[j], tau[j], Ln[j]) for j in range(3)]
    # each single-sample loss is a mean over its own pixels (1/3 of the batch)
    assert np.isclose(loss, sum(w[j] * parts[j][0] for j in range(3)) / 3, rtol=1e-12)
    assert np.allclose(grad, sum(w[j] * parts[j][1] for j in range(3)) / 3, rtol=1e-10, atol=1e-18)
