"""The FED scheme (Eq. 5, one cycle per level) on the GPU against the FP64
oracle, through the C ABI: one cycle with a given conductivity
(kaze_fed_cycle) and the whole scale space, detector and extrema with
params.scheme = KAZE_FED.  The bar is the plain path's: 1e-4 per level on
[0, 1] images, keypoints equal up to the excuse rule."""
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


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (67, 45, 5), (130, 200, 7), (8, 8, 11),
                                      (57, 113, 12)])
def test_fed_cycle_stage(gpu_lib, W, H, seed):
    """One cycle from the oracle's (FP32-rounded) level and conductivity;
    cycle times of the first, a middle and the last level step, and one
    that fits in a single launch."""
    K = gpu_lib
    img = kaze_image(W, H, seed).astype(np.float64)
    L = f32(O.gaussian_smooth(img, 1.6))
    k = O.contrast_factor(L)
    g = f32(O.conductivity_g2(L, k))
    p = K.kaze_default_params()
    p.scheme = K.KAZE_FED
    ws_bytes = K.kaze_workspace_bytes(W, H, p)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    Ld, gd = dev(L), dev(g)
    for T in (0.1, 0.5302, 5.9985, 67.8648):
        K.kaze_fed_cycle(Ld, gd, W, H, T, out, ws, ws_bytes)
        torch.cuda.synchronize()
        ref = O.fed_cycle(L, g, T)
        err = np.max(np.abs(out.cpu().numpy() - ref))
        note(f"[fed_cycle] {W}x{H} seed {seed} T {T} steps {len(O.fed_step_sizes(T))}: "
             f"max|L_gpu - L_orc| = {err:.3e}")
        assert err <= LEVEL_TOL


def test_fed_cycle_constant_and_conservation(gpu_lib):
    """A constant image stays constant; the mean is conserved (no flux
    across the border) up to FP32 rounding."""
    K = gpu_lib
    W, H = 150, 97
    p = K.kaze_default_params()
    p.scheme = K.KAZE_FED
    ws_bytes = K.kaze_workspace_bytes(W, H, p)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    g = dev(np.random.default_rng(3).uniform(0.05, 1.0, size=(H, W)))
    c = torch.full((H, W), 0.375, dtype=torch.float32, device="cuda")
    K.kaze_fed_cycle(c, g, W, H, 33.93, out, ws, ws_bytes)
    torch.cuda.synchronize()
    assert torch.equal(out, c)
    L = dev(kaze_image(W, H, 4))
    K.kaze_fed_cycle(L, g, W, H, 33.93, out, ws, ws_bytes)
    torch.cuda.synchronize()
    m0, m1 = L.double().mean().item(), out.double().mean().item()
    note(f"[fed_cycle] mean {m0:.9f} -> {m1:.9f}")
    assert abs(m1 - m0) < 1e-6


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (103, 71, 6)])
def test_fed_scale_space_vs_oracle(gpu_lib, W, H, seed):
    K = gpu_lib
    img = kaze_image(W, H, seed)
    p = K.kaze_default_params()
    p.scheme = K.KAZE_FED
    kz = K.Kaze(W, H, p, capacity=1 << 16)
    kz.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    lev_o, k_o = O.build_scale_space(img.astype(np.float64), scheme="fed")
    det_o = O.detector_response(lev_o)
    kp_o = O.find_extrema(det_o, 0.001)
    lev_g = kz.levels.cpu().numpy()
    errs = [float(np.abs(lev_g[i] - lev_o[i]).max()) for i in range(len(lev_o))]
    note(f"[fed] {W}x{H} seed {seed}: max|L - L_orc| per level "
         + " ".join("%.1e" % e for e in errs))
    assert float(kz.k.item()) == pytest.approx(k_o, rel=1e-4)
    assert max(errs) <= LEVEL_TOL
    kp_g = kz.keypoints()
    common, bad_g, bad_o = compare_keypoints(kp_g, kp_o, det_o, 0.001)
    note(f"  keypoints {len(kp_g)} / oracle {len(kp_o)}, unexcused {len(bad_g)} + {len(bad_o)}")
    assert not bad_g and not bad_o


def test_fed_differs_from_aos_by_the_scheme_only(gpu_lib):
    """Same image through both schemes: level 0 and k are identical, the
    later levels differ by about what the two FP64 schemes differ by."""
    K = gpu_lib
    W, H = 160, 120
    img = kaze_image(W, H, 8)
    runs = {}
    for name, scheme in (("aos", K.KAZE_AOS), ("fed", K.KAZE_FED)):
        p = K.kaze_default_params()
        p.scheme = scheme
        kz = K.Kaze(W, H, p)
        kz.run(torch.from_numpy(img).cuda())
        torch.cuda.synchronize()
        runs[name] = (kz.levels.cpu().numpy(), float(kz.k.item()))
    la, ka = runs["aos"]
    lf, kf = runs["fed"]
    assert ka == kf and np.array_equal(la[0], lf[0])
    lo_a, _ = O.build_scale_space(img.astype(np.float64))
    lo_f, _ = O.build_scale_space(img.astype(np.float64), scheme="fed")
    d_gpu = np.abs(la - lf).max(axis=(1, 2))
    d_orc = np.abs(lo_a - lo_f).max(axis=(1, 2))
    note("[fed vs aos] GPU " + " ".join("%.1e" % v for v in d_gpu))
    note("[fed vs aos] FP64 " + " ".join("%.1e" % v for v in d_orc))
    assert np.all(np.abs(d_gpu - d_orc) <= 2 * LEVEL_TOL)
