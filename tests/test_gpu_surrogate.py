"""The surrogate's MFMA kernels through the C ABI against the FP64 oracle:
forward pass, loss and parameter gradients, Adam, determinism, and a short
training run on pairs of the plain GPU path."""
import numpy as np
import pytest

from oracle import cnn_oracle as C
from synthetic import kaze_image, surrogate_params
from kaze_parity import note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S(gpu_lib):
    from paper_1706_06750_amd import surrogate
    return surrogate


def planes(n, W, H, seed, exact):
    rng = np.random.default_rng(seed)
    L = np.stack([kaze_image(W, H, seed + j) for j in range(n)]).astype(np.float64)
    g = rng.uniform(0.05, 1.0, size=(n, H, W))
    if exact:
        L, g = C.bf16_round(L), C.bf16_round(g)
    return L.astype(np.float32), g.astype(np.float32)


def params(seed, exact, last_scale=1.0):
    th = surrogate_params(seed, last_scale=last_scale).astype(np.float64)
    if exact:
        th = C.bf16_round(th)
    return th.astype(np.float32)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_forward(S, th, L, g, tau):
    n, H, W = L.shape
    w = S.Weights(th)
    plan = S.Plan(n, W, H, training=False)
    f = plan.forward(w, cuda(L), cuda(g), cuda(np.asarray(tau, np.float32)), add_input=False)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64)


def exact_case(seed, n, W, H, p=0.01):
    """Weights in {-1, 0, 1}, biases and planes on a 1/16 grid, tau / 68 = 1/2:
    every value of the network and of its backward pass is a short binary
    fraction, so BF16 storage and FP32 sums are exact and the GPU must agree
    with the oracle bit for bit.  Returns the parameters, planes, a target
    and tau."""
    rng = np.random.default_rng(seed)
    layers = []
    for ws, bs in C.param_shapes():
        layers.append((rng.choice([-1.0, 0.0, 1.0], size=ws, p=[p / 2, 1 - p, p / 2]),
                       rng.integers(-4, 9, size=bs) / 16.0))
    th = C.flatten(layers)
    L = rng.integers(0, 17, size=(n, H, W)) / 16.0
    g = rng.integers(1, 17, size=(n, H, W)) / 16.0
    Ln = L + rng.integers(-8, 9, size=(n, H, W)) / 16.0 * C.OUT_SCALE * (rng.random((n, H, W)) < 0.3)
    return th, L, g, Ln, np.full(n, 34.0)


def bf16_exact(x):
    return np.array_equal(C.bf16_round(x), x)


@pytest.mark.parametrize("n,W,H", [(2, 37, 29), (1, 70, 75), (3, 16, 8), (1, 9, 100), (1, 130, 33)])
def test_forward_exact_arithmetic(S, n, W, H):
    """Several strips, row chunks and ragged edges; bitwise equal to the oracle."""
    note("[sg] forward %dx%dx%d exact arithmetic" % (n, W, H))
    th, L, g, _, tau = exact_case(10, n, W, H)
    layers = C.unflatten(th)
    X = C.input_planes(L, g, tau)
    for li, (Wt, b) in enumerate(layers):   # precondition: every Z is a BF16 number
        Z = C.conv3x3(X, Wt, b)
        assert bf16_exact(Z), li
        X = np.maximum(Z, 0)
    fo, _ = C.forward(th, L, g, tau, quantized=True)
    fg = run_forward(S, th.astype(np.float32), L.astype(np.float32), g.astype(np.float32), tau)
    note("  max|f| %.3e max|d| %.3e" % (np.abs(fo).max(), np.abs(fg - fo).max()))
    assert np.array_equal(fg, fo)


@pytest.mark.parametrize("n,W,H", [(2, 37, 29), (1, 70, 75), (1, 9, 100)])
def test_forward_bf16_exact_inputs(S, n, W, H):
    """BF16-exact weights and planes: products are exact, and the GPU and the
    quantized oracle differ only through FP32 summation order, which now and
    then moves a stored activation to the neighbouring BF16 number (a CPU
    model with float32 per-tap sums shows the same differences)."""
    note("[sg] forward %dx%dx%d BF16 inputs" % (n, W, H))
    th = params(1, True)
    L, g = planes(n, W, H, 100, True)
    tau = np.array([34.0, 17.0, 68.0][:n])     # tau / 68 exact in BF16
    fg = run_forward(S, th, L, g, tau)
    fo, _ = C.forward(th.astype(np.float64), L, g, tau, quantized=True)
    d = np.abs(fg - fo)
    scale = np.abs(fo).max()
    note("  max|f| %.3e max|d| %.3e mean|d| %.2e frac(|d| > 1e-6 max|f|) %.2e"
         % (scale, d.max(), d.mean(), np.mean(d > 1e-6 * scale)))
    assert d.max() <= 5e-3 * scale
    assert d.mean() <= 2e-4 * scale


@pytest.mark.parametrize("n,W,H", [(2, 53, 41)])
def test_forward_general_inputs(S, n, W, H):
    """Arbitrary FP32 weights and planes: layer 1 is split into three BF16
    terms (relative error ~2^-16), later layers are BF16 by definition."""
    note("[sg] forward %dx%dx%d general inputs" % (n, W, H))
    th = params(2, False)
    L, g = planes(n, W, H, 200, False)
    tau = np.array([1.0604, 47.9876])
    fg = run_forward(S, th, L, g, tau)
    fo, _ = C.forward(th.astype(np.float64), L, g, tau, quantized=True)
    fx, _ = C.forward(th.astype(np.float64), L, g, tau, quantized=False)
    scale = np.abs(fo).max()
    dq = np.abs(fg - fo)
    dx = np.abs(fg - fx)
    note("  vs quantized oracle: max %.3e mean %.3e; vs FP64 network: max %.3e (scale %.3e)"
         % (dq.max(), dq.mean(), dx.max(), scale))
    assert dq.max() <= 2e-2 * scale
    assert dq.mean() <= 3e-3 * scale
    assert dx.max() <= 5e-2 * scale


def run_gradients(S, th, L, g, tau, Ln, reps=1, weights=None):
    n, H, W = L.shape
    w = S.Weights(th)
    plan = S.Plan(n, W, H, training=True)
    args = (cuda(L), cuda(g), cuda(np.asarray(tau, np.float32)), cuda(Ln))
    wt = None if weights is None else cuda(np.asarray(weights, np.float32))
    outs = []
    for _ in range(reps):
        loss = plan.gradients(w, *args, weight=wt)
        torch.cuda.synchronize()
        outs.append((float(loss.item()), w.grad.cpu().numpy().astype(np.float64)))
    return outs


def layer_errors(gg, go):
    out = []
    for (a, b) in zip(C.unflatten(gg), C.unflatten(go)):
        for x, y in zip(a, b):
            out.append(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))
    return out


@pytest.mark.parametrize("n,W,H", [(2, 8, 128), (1, 128, 8)])
def test_gradients_exact_arithmetic(S, n, W, H):
    """n W H a power of two, so dZ of the loss is a short binary fraction as
    well: loss and every parameter gradient bitwise equal to the oracle."""
    note("[sg] gradients %dx%dx%d exact arithmetic" % (n, W, H))
    th, L, g, Ln, tau = exact_case(0, n, W, H)
    wts = np.array([1.0, 0.5])[:n]       # power-of-two loss weights
    layers = C.unflatten(th)
    f, acts = C.forward(th, L, g, tau)
    dZ = (C.OUT_SCALE * 2 * wts[:, None, None] * (f - (Ln - L)) / f.size)[:, None]
    # every dZ is a multiple of 2^-3 OUT_SCALE^2 min(w) / (n W H) (f =
    # OUT_SCALE * a multiple of 1/16) and every activation of 1/16
    unit = 2.0 ** -7 * C.OUT_SCALE ** 2 * wts.min() / f.size
    for li in range(5, -1, -1):          # preconditions: BF16 dZ, exact FP32 sums
        assert bf16_exact(dZ), li
        bound, _ = C.conv3x3_weight_grad(np.abs(acts[li]), np.abs(dZ))
        assert bound.max() / unit < 2 ** 24, li
        if li == 0:
            break
        dZ = C.conv3x3_input_grad(dZ, layers[li][0]) * (acts[li] > 0)
    (lg, gg), = run_gradients(S, th.astype(np.float32), L.astype(np.float32),
                              g.astype(np.float32), tau, Ln.astype(np.float32), weights=wts)
    lo, go, _ = C.loss_and_grad(th, L, g, tau, Ln, quantized=True, weights=wts)
    note("  loss %.6e / %.6e; nonzero gradients %d; max|diff| %.3e"
         % (lg, lo, int(np.count_nonzero(go)), np.abs(gg - go).max()))
    assert np.count_nonzero(go) > 1000
    assert lg == lo
    assert np.array_equal(gg, go)


@pytest.mark.parametrize("n,W,H", [(2, 33, 20), (1, 64, 70)])
def test_gradients_bf16_exact_inputs(S, n, W, H):
    note("[sg] gradients %dx%dx%d BF16 inputs" % (n, W, H))
    th = params(3, True, last_scale=1.0)
    L, g = planes(n, W, H, 300, True)
    Ln = (L + 0.02 * np.sin(np.arange(L.size).reshape(L.shape))).astype(np.float32)
    tau = np.array([34.0, 17.0][:n])
    (lg, gg), = run_gradients(S, th, L, g, tau, Ln)
    lo, go, _ = C.loss_and_grad(th.astype(np.float64), L, g, tau, Ln, quantized=True)
    errs = layer_errors(gg, go)
    note("  loss %.6e / %.6e; per-tensor relative errors %s"
         % (lg, lo, " ".join("%.1e" % e for e in errs)))
    assert abs(lg - lo) <= 1e-3 * lo
    assert max(errs) <= 1e-2


def test_gradients_general_inputs_vs_fp64(S):
    """Against the quantized reading and against the unrounded FP64 network."""
    n, W, H = 2, 40, 36
    note("[sg] gradients %dx%dx%d general inputs" % (n, W, H))
    th = params(4, False, last_scale=1.0)
    L, g = planes(n, W, H, 400, False)
    Ln = (L + 0.03 * np.cos(np.arange(L.size).reshape(L.shape) * 0.37)).astype(np.float32)
    tau = np.array([2.1208, 23.9938])
    wts = 1.0 / tau                      # the training weights
    (lg, gg), = run_gradients(S, th, L, g, tau, Ln, weights=wts.astype(np.float32))
    wq = wts.astype(np.float32).astype(np.float64)
    lo, go, _ = C.loss_and_grad(th.astype(np.float64), L, g, tau, Ln, quantized=True, weights=wq)
    lx, gx, _ = C.loss_and_grad(th.astype(np.float64), L, g, tau, Ln, quantized=False, weights=wq)
    eq, ex = layer_errors(gg, go), layer_errors(gg, gx)
    note("  quantized: loss %.3e/%.3e max tensor err %.2e; FP64: loss %.3e max err %.2e"
         % (lg, lo, max(eq), lx, max(ex)))
    assert abs(lg - lo) <= 1e-3 * lo
    assert max(eq) <= 2e-2
    assert max(ex) <= 1e-1
    # the gradient points the same way as the exact FP64 gradient
    cos = float(np.dot(gg, gx) / (np.linalg.norm(gg) * np.linalg.norm(gx)))
    assert cos > 0.999


def test_deterministic(S):
    th = params(5, False)
    L, g = planes(2, 45, 38, 500, False)
    Ln = (L * 0.9 + 0.05).astype(np.float32)
    tau = np.array([4.2415, 0.5302])
    outs = run_gradients(S, th, L, g, tau, Ln, reps=2)
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])


def test_adam_matches_oracle(S):
    rng = np.random.default_rng(6)
    th = params(6, False)
    w = S.Weights(th)
    m = np.zeros(th.size)
    v = np.zeros(th.size)
    ref = th.astype(np.float64)
    for step in (1, 2, 3):
        gr = (rng.normal(size=th.size) * 10.0 ** rng.integers(-6, 0, size=th.size)).astype(np.float32)
        w.grad.copy_(torch.from_numpy(gr))
        w.adam(lr=1e-3)
        ref, m, v = C.adam_step(ref, gr.astype(np.float64), m, v, step, lr=1e-3)
    torch.cuda.synchronize()
    got = w.params.cpu().numpy().astype(np.float64)
    # three updates of at most lr each; FP32 arithmetic
    assert np.max(np.abs(got - ref)) <= 3e-3 * 1e-4 + 4 * np.abs(ref).max() * 2 ** -24


def test_training_lowers_the_loss(S, gpu_lib):
    """A few hundred Adam steps on level pairs of the plain GPU path."""
    K = gpu_lib
    W = H = 64
    nimg = 4
    kz = K.Kaze(W, H)
    Ls, gs, Lns, taus = [], [], [], []
    sched = K.kaze_schedule(kz.p)
    for j in range(nimg):
        img = torch.from_numpy(kaze_image(W, H, 700 + j)).cuda()
        kz.run(img)
        k = float(kz.k.item())
        for i in range(1, 6):
            gbuf = torch.empty((H, W), device="cuda")
            K.kaze_conductivity(kz.levels[i - 1], W, H, kz.p, k, gbuf)
            Ls.append(kz.levels[i - 1].clone())
            gs.append(gbuf)
            Lns.append(kz.levels[i].clone())
            taus.append(sched[i]["tau"])
    L = torch.stack(Ls)
    g = torch.stack(gs)
    Ln = torch.stack(Lns)
    tau = torch.tensor(taus, dtype=torch.float32, device="cuda")
    w = S.Weights(surrogate_params(7))
    plan = S.Plan(L.shape[0], W, H, training=True)
    no_step = float(((Ln - L) ** 2).mean().item())
    losses = []
    for it in range(300):
        loss = plan.gradients(w, L, g, tau, Ln)
        if it % 50 == 0 or it == 299:
            losses.append(float(loss.item()))
        w.adam(lr=2e-3)
    torch.cuda.synchronize()
    note("[sg] training losses %s (no step: %.3e)" % (" ".join("%.3e" % v for v in losses), no_step))
    assert losses[-1] < 0.5 * losses[0]
    assert losses[-1] < no_step
