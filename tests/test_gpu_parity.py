"""GPU path vs the FP64 oracle, through the C ABI.

Stage-isolated tests feed each GPU stage the oracle's own (FP32-rounded)
inputs, so they measure one stage's FP32 error; end-to-end tests run the
whole path and apply the per-level bound LEVEL_TOL and the keypoint rule.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image
from kaze_parity import LEVEL_TOL, compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def run_gpu(K, img, params=None, capacity=1 << 16, stream=None):
    H, W = img.shape
    kz = K.Kaze(W, H, params, capacity=capacity)
    x = dev(img)
    kz.run(x, stream)
    torch.cuda.synchronize()
    return kz


def run_oracle(img, **kw):
    lev, k = O.build_scale_space(img.astype(np.float64), **kw)
    det = O.detector_response(lev)
    return lev, k, det


def det_tolerance(level_err, sn2, s):
    """Bound on |det_gpu - det_orc| given the level error eps: each second
    derivative D_s D_s moves by at most eps/s^2 and is at most 1/(2 s^2) in
    size for values in [0, 1], so det = sn^2 (Lxx Lyy - Lxy^2) moves by at
    most sn^2 * 3 * (eps/s^2) * (1/(2 s^2)) * 2 (+ eps^2 terms); a floor of
    1e-7 sn^2 covers FP32 rounding of the detector itself."""
    return sn2 * (3.0 * level_err / s ** 4 + 1e-7)


def g_tolerance(k, radius=3):
    """FP32 bound for the conductivity of an image in [0, 1]: each of the
    two Gaussian passes ((2r+1) taps) and the tap rounding leave an absolute
    error of at most (2r+1) u per pass in the smoothed image (u = 2^-24);
    the Scharr kernel (sum of |taps| = 1) passes it on to each gradient
    component, so |d|grad|| <= 2 * 2 (2r+1) u; and |dg/d|grad|| <= 0.65/k
    for g2 (maximum of 2m/k^2/(1+m^2/k^2)^2 at m = k/sqrt(3))."""
    u = 2.0 ** -24
    return 0.65 / k * 4 * (2 * radius + 1) * u


# ---------------------------------------------------------------- stages
@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (67, 45, 5), (1920, 1200, 2)])
def test_conductivity_stage(gpu_lib, W, H, seed):
    K = gpu_lib
    note(f"[conductivity] {W}x{H} seed {seed}")
    img = kaze_image(W, H, seed).astype(np.float64)
    L = f32(O.gaussian_smooth(img, 1.6))
    k = O.contrast_factor(L)
    p = K.kaze_default_params()
    g = torch.empty((H, W), dtype=torch.float32, device="cuda")
    K.kaze_conductivity(dev(L), W, H, p, k, g)
    torch.cuda.synchronize()
    k32 = float(np.float32(k))
    ref = O.conductivity_g2(L, k32)
    err = np.max(np.abs(g.cpu().numpy() - ref))
    note(f"  max|g_gpu - g_orc| = {err:.3e} (k = {k32:.4g}, bound {g_tolerance(k32):.2e})")
    assert err < g_tolerance(k32)


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (67, 45, 5), (130, 97, 6), (9, 13, 3)])
def test_conductivity_equals_fused_reduction(gpu_lib, W, H, seed):
    """kaze_conductivity runs the AOS reduction's own band code, so its g
    equals, bit for bit, the g plane that the last fused reduction of a
    scale-space build (level N-1, from level N-2 and the build's k) leaves in
    the first region of the plain workspace."""
    K = gpu_lib
    img = kaze_image(W, H, seed)
    kz = K.Kaze(W, H)
    kz.scale_space(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    g_fused = kz.ws[: W * H * 4].view(torch.float32).reshape(H, W).clone()
    g = torch.empty((H, W), dtype=torch.float32, device="cuda")
    K.kaze_conductivity(kz.levels[kz.N - 2].contiguous(), W, H, kz.p, float(kz.k.item()), g)
    torch.cuda.synchronize()
    note(f"[conductivity] {W}x{H}: standalone vs fused g, max|d| "
         f"{(g - g_fused).abs().max().item():.1e}")
    assert torch.equal(g, g_fused)


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (67, 45, 5), (1920, 1200, 2),
                                      (130, 1100, 7), (64, 2100, 8), (4000, 20, 9),
                                      (4096, 9, 10), (8, 8, 11)])
def test_aos_step_stage(gpu_lib, W, H, seed):
    K = gpu_lib
    img = kaze_image(W, H, seed).astype(np.float64)
    L = f32(O.gaussian_smooth(img, 1.6))
    k = O.contrast_factor(L)
    g = f32(O.conductivity_g2(L, k))
    p = K.kaze_default_params()
    ws_bytes = K.kaze_workspace_bytes(W, H, p)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    Ld, gd = dev(L), dev(g)
    for tau in (0.5302, 5.9985, 67.8648):
        note(f"[aos_step] {W}x{H} seed {seed} tau {tau}")
        K.kaze_aos_step(Ld, gd, W, H, tau, out, ws, ws_bytes)
        torch.cuda.synchronize()
        ref = O.aos_step(L, g, tau)
        err = np.max(np.abs(out.cpu().numpy() - ref))
        note(f"  max|L_gpu - L_orc| = {err:.3e}")
        assert err < 2e-6


def test_detector_stage(gpu_lib):
    K = gpu_lib
    W, H = 320, 240
    note(f"[detector] {W}x{H}")
    lev, _ = O.build_scale_space(kaze_image(W, H, 1).astype(np.float64))
    lev32 = f32(lev)
    p = K.kaze_default_params()
    det = torch.empty(lev.shape, dtype=torch.float32, device="cuda")
    K.kaze_detector_response(dev(lev32), W, H, p, det)
    torch.cuda.synchronize()
    ref = O.detector_response(lev32)
    d = det.cpu().numpy()
    for i in range(lev.shape[0]):
        err = np.max(np.abs(d[i] - ref[i]))
        assert err < 1e-8, (i, err)


@pytest.mark.parametrize("W,H,sigma0", [(200, 150, 4.0), (200, 150, 4.5), (70, 66, 4.0),
                                         (40, 20, 4.5), (33, 12, 4.5), (61, 9, 1.6)])
def test_detector_stage_all_steps(gpu_lib, W, H, sigma0):
    """The detector on every Scharr step it accepts (sigma0 4.0 gives steps
    4, 5, 6, 7 in each octave, 4.5 gives 5, 5, 6, 8) and on every form of
    its strips: bands of 64 rows, bands of 8 rows (70x66, 40x20), the
    per-pixel form of images too low for a band (33x12 at steps above 4,
    61x9), widths of one strip and of several with the last one aligned to
    the image end.  Inputs are smooth random levels.  Bound per level: the
    FP32 error of det = sigma_n^2 (Lxx Lyy - Lxy^2) is a few units of the
    second derivatives' rounding times their size (the products cancel, so
    |det| itself is no scale): 1e-6 sigma_n^2 max(|Lxx| + |Lyy| + 2 |Lxy|),
    from the oracle's own derivatives."""
    from scipy.ndimage import gaussian_filter
    K = gpu_lib
    note(f"[detector] {W}x{H} sigma0 {sigma0}")
    p = K.kaze_default_params(sigma0=sigma0)
    N = K.kaze_num_levels(p)
    rng = np.random.default_rng(W * 1000 + H)
    lev = np.stack([gaussian_filter(rng.random((H, W)), 1.5, mode="reflect") for _ in range(N)])
    lev32 = f32(lev)
    det = torch.empty(lev.shape, dtype=torch.float32, device="cuda")
    K.kaze_detector_response(dev(lev32), W, H, p, det)
    torch.cuda.synchronize()
    ref = O.detector_response(lev32, sigma0=sigma0)
    d = det.cpu().numpy()
    for lv in O.level_schedule(sigma0, 4, 4):
        i = lv["i"]
        sn = lv["sigma"] / 2.0 ** lv["o"]
        st = O.derivative_step(sn)
        Lx, Ly = O.scharr_dx(lev32[i], st), O.scharr_dy(lev32[i], st)
        scale = np.max(np.abs(O.scharr_dx(Lx, st)) + np.abs(O.scharr_dy(Ly, st))
                       + 2 * np.abs(O.scharr_dy(Lx, st)))
        err = np.max(np.abs(d[i] - ref[i]))
        assert err <= 1e-6 * sn * sn * scale, (i, st, err, sn * sn * scale)


@pytest.mark.parametrize("W,H,sigma0", [(320, 240, 1.6), (130, 70, 1.6), (200, 150, 4.0),
                                         (40, 20, 4.5), (33, 12, 4.5)])
def test_detector_mirror_equivariant(gpu_lib, W, H, sigma0):
    """det = sigma_n^2 (Lxx Lyy - Lxy^2) is unchanged by a vertical mirror of
    the levels (Lxy changes sign and is squared).  In the kernels' FP32
    arithmetic it holds bit for bit: vertical differences change sign
    exactly and the vertical Scharr sums are symmetric in their outer rows,
    so a mistake in the reflection at the bottom border that the top does
    not share, or an asymmetric vertical stencil, fails it.  Cases: bands
    of 32 rows with an aligned last band (320x240, 130x70), steps 4-7
    (200x150), bands of 8 rows (40x20) and the per-pixel form (33x12)."""
    from scipy.ndimage import gaussian_filter
    K = gpu_lib
    note(f"[detector mirror] {W}x{H} sigma0 {sigma0}")
    p = K.kaze_default_params(sigma0=sigma0)
    N = K.kaze_num_levels(p)
    rng = np.random.default_rng(W * 7 + H)
    lev = f32(np.stack([gaussian_filter(rng.random((H, W)), 1.5, mode="reflect")
                        for _ in range(N)]))
    det = torch.empty(lev.shape, dtype=torch.float32, device="cuda")
    det_m = torch.empty(lev.shape, dtype=torch.float32, device="cuda")
    K.kaze_detector_response(dev(lev), W, H, p, det)
    K.kaze_detector_response(dev(np.ascontiguousarray(lev[:, ::-1, :])), W, H, p, det_m)
    torch.cuda.synchronize()
    assert torch.equal(det_m.flip(1), det)


# ---------------------------------------------------------------- end to end
def check_end_to_end(K, W, H, seed, params=None, oracle_kw=None):
    note(f"[end-to-end] {W}x{H} seed {seed} params {params and dict((f, getattr(params, f)) for f, _ in params._fields_)}")
    img = kaze_image(W, H, seed)
    kz = run_gpu(K, img, params)
    lev_o, k_o, det_o = run_oracle(img, **(oracle_kw or {}))
    k_g = float(kz.k.item())
    note(f"  k gpu {k_g:.9g} oracle {k_o:.9g}")
    assert k_g == pytest.approx(k_o, rel=1e-4)
    lev_g = kz.levels.cpu().numpy()
    det_g = kz.det.cpu().numpy()
    sched = K.kaze_schedule(kz.p)
    worst = 0.0
    for i in range(kz.N):
        e = float(np.max(np.abs(lev_g[i] - lev_o[i])))
        de = float(np.max(np.abs(det_g[i] - det_o[i])))
        sn2 = sched[i]["sigma_norm"] ** 2
        note(f"  level {i:2d}: max|dL| {e:.2e}  max|ddet| {de:.2e}")
        worst = max(worst, e)
        assert e <= LEVEL_TOL, (i, e)
        assert de <= det_tolerance(e, sn2, sched[i]["deriv_step"]), (i, de)
    kp_g = kz.keypoints()
    thr = kz.p.det_threshold
    kp_o = O.find_extrema(det_o, thr)
    common, bad_g, bad_o = compare_keypoints(kp_g, kp_o, det_o, thr)
    note(f"  keypoints gpu {len(kp_g)} oracle {len(kp_o)} common {common} "
         f"unexcused gpu-only {bad_g[:5]} oracle-only {bad_o[:5]}")
    assert not bad_g and not bad_o
    return worst


@pytest.mark.parametrize("sigma_cond", [0.3, 0.6, 1.3])
def test_other_conductivity_radii(gpu_lib, sigma_cond):
    """sigma_cond of Gaussian radius 1, 2 and 4 (ceil(3 sigma); the default
    1.0 has 3): the whole path against the oracle, and the standalone
    conductivity equal, bit for bit, to the g of the fused reduction."""
    K = gpu_lib
    p = K.kaze_default_params(sigma_cond=sigma_cond)
    check_end_to_end(K, 160, 120, 4, p, dict(sigma_cond=sigma_cond))
    W, H = 130, 97
    kz = K.Kaze(W, H, p)
    kz.scale_space(torch.from_numpy(kaze_image(W, H, 6)).cuda())
    torch.cuda.synchronize()
    g_fused = kz.ws[: W * H * 4].view(torch.float32).reshape(H, W).clone()
    g = torch.empty((H, W), dtype=torch.float32, device="cuda")
    K.kaze_conductivity(kz.levels[kz.N - 2].contiguous(), W, H, p, float(kz.k.item()), g)
    torch.cuda.synchronize()
    assert torch.equal(g, g_fused)


@pytest.mark.parametrize("sigma0", [1.0, 2.4, 3.0])
def test_other_detector_steps(gpu_lib, sigma0):
    """sigma0 whose levels take Scharr steps {1, 2} (one launch for both),
    {2, 3, 4} (one launch per step) and {3, 4, 5} (step 5 on the
    per-position detector): levels, det and keypoints against the oracle,
    and the batch (whose detector also writes the threshold masks) equal to
    the single-image calls."""
    K = gpu_lib
    W, H = 160, 120
    p = K.kaze_default_params(sigma0=sigma0)
    img = kaze_image(W, H, 5)
    kz = run_gpu(K, img, p)
    lev_o, k_o = O.build_scale_space(img.astype(np.float64), sigma0=sigma0)
    det_o = O.detector_response(lev_o, sigma0=sigma0)
    sched = K.kaze_schedule(kz.p)
    note(f"[detector steps] sigma0 {sigma0}: steps {sorted({s['deriv_step'] for s in sched})}")
    assert float(kz.k.item()) == pytest.approx(k_o, rel=1e-4)
    lev_g, det_g = kz.levels.cpu().numpy(), kz.det.cpu().numpy()
    for i in range(kz.N):
        e = float(np.max(np.abs(lev_g[i] - lev_o[i])))
        de = float(np.max(np.abs(det_g[i] - det_o[i])))
        assert e <= LEVEL_TOL, (i, e)
        assert de <= det_tolerance(e, sched[i]["sigma_norm"] ** 2, sched[i]["deriv_step"]), (i, de)
    thr = kz.p.det_threshold
    common, bad_g, bad_o = compare_keypoints(kz.keypoints(), O.find_extrema(det_o, thr), det_o, thr)
    note(f"  keypoints common {common}, unexcused {len(bad_g)} + {len(bad_o)}")
    assert not bad_g and not bad_o
    kb = K.KazeBatch([(W, H), (67, 45)], params=p, shape=0)
    kb.inputs[0].copy_(torch.from_numpy(img))
    kb.inputs[1].copy_(torch.from_numpy(kaze_image(67, 45, 6)))
    kb.run()
    torch.cuda.synchronize()
    assert torch.equal(kb.det[0], kz.det)
    assert np.array_equal(kb.keypoints(0), kz.keypoints())
    kb.close()


def test_end_to_end_320x240(gpu_lib):
    check_end_to_end(gpu_lib, 320, 240, 1)


def test_end_to_end_1920x1200(gpu_lib):
    check_end_to_end(gpu_lib, 1920, 1200, 2)


@pytest.mark.parametrize("W,H,seed", [(8, 8, 21), (9, 13, 22), (67, 45, 23), (130, 1100, 24),
                                      (64, 2100, 25), (4000, 20, 26), (4096, 9, 27),
                                      (1000, 33, 28)])
def test_end_to_end_ragged_and_extreme_shapes(gpu_lib, W, H, seed):
    check_end_to_end(gpu_lib, W, H, seed)


@pytest.mark.parametrize("nbins", [1, 37, 1000, 4096])
def test_histogram_bin_counts(gpu_lib, nbins):
    """The contrast factor for 1 to 4096 bins (the block and global
    histograms, the copies kselect sums): within one bin width of the
    oracle's k (the FP32 and FP64 gradients may put a pixel on either side of
    a bin edge)."""
    K = gpu_lib
    W, H = 320, 240
    img = kaze_image(W, H, 4)
    kz = K.Kaze(W, H, K.kaze_default_params(k_bins=nbins))
    kz.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    L0 = O.gaussian_smooth(img.astype(np.float64), 1.6)
    k_o = O.contrast_factor(L0, nbins=nbins)
    hmax = float(O.gradient_magnitude(L0, 1.0).max())
    k_g = float(kz.k.item())
    note(f"[histogram] {nbins} bins: k {k_g:.6e} oracle {k_o:.6e} bin width {hmax / nbins:.2e}")
    assert abs(k_g - k_o) <= hmax / nbins * 1.001


def test_k_override_and_g1(gpu_lib):
    K = gpu_lib
    p = K.kaze_default_params(k_override=0.004)
    check_end_to_end(K, 320, 240, 3, p, dict(k=float(np.float32(0.004))))
    p = K.kaze_default_params(diffusivity=K.KAZE_G1)
    check_end_to_end(K, 320, 240, 4, p, dict(diffusivity="g1"))


def test_constant_image(gpu_lib):
    K = gpu_lib
    note("[constant] 96x80")
    img = np.full((80, 96), 0.4321, dtype=np.float32)
    kz = run_gpu(K, img)
    assert float(kz.k.item()) == 1.0
    lev = kz.levels.cpu().numpy()
    assert np.max(np.abs(lev - lev[0, 40, 40])) == 0.0
    assert abs(lev[0, 40, 40] - 0.4321) < 1e-6
    assert np.max(np.abs(kz.det.cpu().numpy())) == 0.0
    assert int(kz.count.item()) == 0


def test_deterministic_and_stream_ordered(gpu_lib):
    K = gpu_lib
    note("[determinism] 640x480 seed 31, default and side stream")
    img = kaze_image(640, 480, 31)
    a = run_gpu(K, img)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        kz = K.Kaze(640, 480)
        x = dev(img)
        kz.run(x, s)
    s.synchronize()
    assert torch.equal(a.levels, kz.levels)
    assert torch.equal(a.det, kz.det)
    assert np.array_equal(a.keypoints(), kz.keypoints())


def test_capacity_overflow(gpu_lib):
    K = gpu_lib
    note("[capacity] 320x240 seed 1 capacity 1")
    img = kaze_image(320, 240, 1)
    full = run_gpu(K, img)
    n = int(full.count.item())
    assert n > 1
    kps = torch.full((8, 4), -7, dtype=torch.int32, device="cuda")
    count = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    K.kaze_find_extrema(full.det, 320, 240, full.p, kps, 1, count)
    torch.cuda.synchronize()
    assert int(count.item()) == n
    rows = kps.cpu().numpy()
    assert (rows[1:] == -7).all()            # nothing written past the capacity
    first = (int(rows[0, 2]), int(rows[0, 1]), int(rows[0, 0]))
    assert first in {tuple(int(v) for v in r[:3]) for r in full.keypoints()}
