"""The exact cross-level extrema test (Sec. II-B, Sec. III-B, Sec. IV) on
the GPU against the FP64 oracle, through the C ABI: params.extrema_window =
KAZE_WINDOW_SIGMA in kaze_find_extrema, the whole single-image path and the
batched form.

Stage: both sides compare the same FP32 responses (and the FP32 threshold),
so the sets must be equal.  End to end: the keypoint rule of the plain path,
with neighbours taken over the cross-level window."""
import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image
from kaze_parity import compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def radii_of(p):
    return [O.cross_level_radius(s["sigma"])
            for s in O.level_schedule(p.sigma0, p.octaves, p.sublevels)]


def sigma_params(K):
    p = K.kaze_default_params()
    p.extrema_window = K.KAZE_WINDOW_SIGMA
    return p


def as_set(kps):
    return {tuple(int(v) for v in r[:3]) for r in kps}


def gpu_extrema(K, det32, p, capacity=1 << 16):
    N, H, W = det32.shape
    kps = torch.empty((capacity, 4), dtype=torch.int32, device="cuda")
    count = torch.empty(1, dtype=torch.int32, device="cuda")
    K.kaze_find_extrema(torch.from_numpy(det32).cuda(), W, H, p, kps, capacity, count)
    torch.cuda.synchronize()
    n = int(count.item())
    assert n <= capacity
    rows = kps[:n].cpu().numpy()
    return {(int(r[2]), int(r[1]), int(r[0])) for r in rows}


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (200, 130, 2)])
def test_window_stage_equals_oracle(gpu_lib, W, H, seed):
    K = gpu_lib
    p = sigma_params(K)
    lev, _ = O.build_scale_space(kaze_image(W, H, seed).astype(np.float64))
    det32 = O.detector_response(lev).astype(np.float32)
    thr = float(np.float32(p.det_threshold))
    ref = as_set(O.find_extrema(det32.astype(np.float64), thr, radii_of(p)))
    approx = as_set(O.find_extrema(det32.astype(np.float64), thr))
    got = gpu_extrema(K, det32, p)
    note(f"[window] {W}x{H} seed {seed}: exact {len(got)} (oracle {len(ref)}), "
         f"3x3x3 {len(approx)}")
    assert got == ref and len(ref) > 0


def test_window_stage_random_responses(gpu_lib):
    """Random responses with threshold 0: many candidates, windows clipped
    at every border, 20 levels so that the half-sides reach 20."""
    K = gpu_lib
    p = sigma_params(K)
    p.octaves, p.sublevels = 5, 4
    rng = np.random.default_rng(5)
    N, H, W = 20, 45, 67
    det32 = rng.normal(0, 1, size=(N, H, W)).astype(np.float32)
    det32 += np.linspace(0, 3, N, dtype=np.float32)[::-1, None, None] * \
        rng.random((N, 1, 1), dtype=np.float32)
    radii = radii_of(p)
    assert max(radii) >= 15
    ref = as_set(O.find_extrema(det32.astype(np.float64), 0.0, radii))
    got = gpu_extrema(K, det32, p)
    note(f"[window] random {N}x{H}x{W}: {len(got)} extrema, radii {radii}")
    assert got == ref and len(ref) > 10


@pytest.mark.parametrize("W,H,seed", [(320, 240, 1), (131, 97, 4)])
def test_window_end_to_end(gpu_lib, W, H, seed):
    K = gpu_lib
    p = sigma_params(K)
    img = kaze_image(W, H, seed)
    kz = K.Kaze(W, H, p)
    kz.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    kp_g = kz.keypoints()
    lev, _ = O.build_scale_space(img.astype(np.float64))
    det_o = O.detector_response(lev)
    radii = radii_of(p)
    kp_o = O.find_extrema(det_o, p.det_threshold, radii)
    common, bad_g, bad_o = compare_keypoints(kp_g, kp_o, det_o, p.det_threshold, radii)
    note(f"[window e2e] {W}x{H} seed {seed}: gpu {len(kp_g)} oracle {len(kp_o)} common {common}")
    assert not bad_g and not bad_o
    # the exact set is a subset of the 3x3x3 set of the same run
    approx = K.Kaze(W, H)
    approx.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    assert torch.equal(approx.det, kz.det)
    assert as_set(kp_g) <= as_set(approx.keypoints())


def test_window_batch_equals_single(gpu_lib):
    K = gpu_lib
    p = sigma_params(K)
    sizes = [(320, 240), (67, 45), (200, 130)]
    kb = K.KazeBatch(sizes, params=p, shape=0)
    imgs = [kaze_image(W, H, 60 + j) for j, (W, H) in enumerate(sizes)]
    for x, im in zip(kb.inputs, imgs):
        x.copy_(torch.from_numpy(im))
    kb.run()
    torch.cuda.synchronize()
    for j, im in enumerate(imgs):
        H, W = im.shape
        kz = K.Kaze(W, H, p)
        kz.run(torch.from_numpy(im).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(kb.keypoints(j), kz.keypoints())
    kb.close()
