"""Batched form through the C ABI: many images of uneven sizes, one launch per
phase, replayed from a captured hipGraph, with the tile shape of the line
solves chosen by the autotuner."""
import numpy as np
import pytest

import oracle as O
from synthetic import batch_sizes, kaze_image
from kaze_parity import LEVEL_TOL, compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# ragged sizes covering partial tiles of every shape (60 wide, 32 or 64
# high; row chunks of 30, column chunks of 32), images narrower than a row
# chunk and taller than wide, an exact multiple of the tile
SIZES = [(67, 45), (320, 240), (200, 130), (130, 260), (64, 64), (9, 13), (120, 96), (31, 33)]


def single(K, img):
    H, W = img.shape
    kz = K.Kaze(W, H)
    kz.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    return kz


def make_batch(K, sizes, seeds, shape, **kw):
    kb = K.KazeBatch(sizes, shape=shape, **kw)
    imgs = [kaze_image(W, H, s) for (W, H), s in zip(sizes, seeds)]
    for x, im in zip(kb.inputs, imgs):
        x.copy_(torch.from_numpy(im))
    return kb, imgs


def _same_arithmetic(K, a, b):
    """Shapes with the same chunk lengths, interface chunks per lane and
    sweep lanes per chunk evaluate the same arithmetic."""
    x, y = K.AOS_SHAPES[a], K.AOS_SHAPES[b]
    return all(x[k] == y[k] for k in ("row_chunk", "col_chunk", "iface_m", "chunk_lanes"))


@pytest.mark.parametrize("shape", range(6))
def test_batch_matches_single_image_path(gpu_lib, shape):
    """Every launch shape against the single-image calls (default shape 0 for
    these sizes): bitwise where the chunk lengths and interface lanes are
    the same, else within FP32 rounding of the two elimination orders
    (levels 1e-5, a tenth of the oracle tolerance) with the keypoint sets
    equal up to points the excuse rule covers."""
    K = gpu_lib
    assert len(K.AOS_SHAPES) == 6
    note(f"[batch] shape {K.shape_label(shape)} sizes {SIZES}")
    kb, imgs = make_batch(K, SIZES, range(40, 40 + len(SIZES)), shape)
    # a small batch runs the detector after the steps
    assert kb.det_levels_in_segment == 0
    kb.run()
    torch.cuda.synchronize()
    exact = _same_arithmetic(K, shape, 0)
    for j, im in enumerate(imgs):
        ref = single(K, im)
        assert float(kb.k[j].item()) == float(ref.k.item())
        assert torch.equal(kb.levels[j][0], ref.levels[0])
        dl = (kb.levels[j] - ref.levels).abs().max().item()
        dd = (kb.det[j] - ref.det).abs().max().item()
        note(f"  image {j} {SIZES[j]}: max|dL| {dl:.2e} max|ddet| {dd:.2e}")
        if exact:
            assert dl == 0.0 and dd == 0.0
            assert np.array_equal(kb.keypoints(j), ref.keypoints())
        else:
            assert dl <= 1e-5, (j, dl)
            det_ref = ref.det.cpu().numpy().astype(np.float64)
            _, bad_b, bad_r = compare_keypoints(kb.keypoints(j), ref.keypoints(), det_ref, 0.001)
            assert not bad_b and not bad_r, (j, bad_b, bad_r)
    kb.close()


def test_batch_graph_replays_match_eager(gpu_lib):
    K = gpu_lib
    note("[batch] graph replays vs eager, shape 1")
    kb, _ = make_batch(K, SIZES, range(60, 60 + len(SIZES)), 1)
    kb.run(eager=True)
    torch.cuda.synchronize()
    ref_lv = [t.clone() for t in kb.levels]
    ref_det = [t.clone() for t in kb.det]
    ref_cnt = [int(c.item()) for c in kb.count]
    for r in range(3):
        for t in kb.levels:
            t.fill_(-1.0)
        kb.run()
        torch.cuda.synchronize()
        for j in range(len(SIZES)):
            assert torch.equal(kb.levels[j], ref_lv[j]), (r, j)
            assert torch.equal(kb.det[j], ref_det[j]), (r, j)
            assert int(kb.count[j].item()) == ref_cnt[j], (r, j)
    kb.close()


@pytest.mark.parametrize("sigma0", [0.6, 3.2])
def test_batch_detector_at_other_schedules(gpu_lib, sigma0):
    """Schedules with other Scharr steps (sigma0 0.6: every step 1; sigma0
    3.2: steps 3 to 5, two detector launches): a small batch's graph runs,
    eager runs and the single-image calls agree bitwise, keypoints
    included."""
    K = gpu_lib
    p = K.kaze_default_params(sigma0=sigma0)
    sizes = SIZES[:4]
    note(f"[batch] sigma0 {sigma0}: sizes {sizes}")
    kb, imgs = make_batch(K, sizes, range(120, 124), 0, params=p)
    assert kb.det_levels_in_segment == 0
    kb.run(eager=True)
    torch.cuda.synchronize()
    ref_det = [t.clone() for t in kb.det]
    ref_cnt = [int(c.item()) for c in kb.count]
    for t in kb.det:
        t.fill_(-1.0)
    kb.run()
    torch.cuda.synchronize()
    for j, im in enumerate(imgs):
        assert torch.equal(kb.det[j], ref_det[j]), j
        assert int(kb.count[j].item()) == ref_cnt[j], j
        H, W = im.shape
        kz = K.Kaze(W, H, params=p)
        kz.run(torch.from_numpy(im).cuda())
        torch.cuda.synchronize()
        assert torch.equal(kb.levels[j], kz.levels), j
        assert torch.equal(kb.det[j], kz.det), j
        assert np.array_equal(kb.keypoints(j), kz.keypoints()), j
    kb.close()


def test_autotuner_and_cache(gpu_lib, tmp_path):
    K = gpu_lib
    cache = str(tmp_path / "tune.json")
    note("[batch] autotune")
    kb = K.KazeBatch(SIZES, shape="auto", tune_cache=cache)
    assert kb.shape in range(len(K.AOS_SHAPES))
    assert kb.tune_ms is not None and min(m for m in kb.tune_ms if m > 0) > 0
    note(f"  ms per shape {kb.tune_ms} -> {K.shape_label(kb.shape)}")
    kb.close()
    kb2 = K.KazeBatch(SIZES, shape="auto", tune_cache=cache)
    assert kb2.shape == kb.shape
    kb2.close()


def test_uneven_batch_images_vs_oracle(gpu_lib):
    """Two images of the 64-image uneven workload, inside a batch of four,
    against the FP64 oracle."""
    K = gpu_lib
    sizes = batch_sizes(64, 3, 640, 1920, 480, 1200)[:4]
    seeds = [3000 + j for j in range(4)]
    note(f"[batch] uneven workload images {sizes}")
    kb, imgs = make_batch(K, sizes, seeds, "auto")
    kb.run()
    torch.cuda.synchronize()
    for j in (0, 3):
        lev_o, k_o = O.build_scale_space(imgs[j].astype(np.float64))
        det_o = O.detector_response(lev_o)
        lev_g = kb.levels[j].cpu().numpy()
        err = max(float(np.max(np.abs(lev_g[i] - lev_o[i]))) for i in range(kb.N))
        kp_o = O.find_extrema(det_o, 0.001)
        common, bad_g, bad_o = compare_keypoints(kb.keypoints(j), kp_o, det_o, 0.001)
        note(f"  image {j} {sizes[j]}: k {kb.k[j].item():.6g}/{k_o:.6g} worst level err "
             f"{err:.2e} keypoints {common}/{len(kp_o)}")
        assert float(kb.k[j].item()) == pytest.approx(k_o, rel=1e-4)
        assert err <= LEVEL_TOL
        assert not bad_g and not bad_o
    kb.close()


def test_full_uneven_batch_equals_single_image_calls(gpu_lib):
    """The whole 64-image uneven workload (W in [640, 1920], H in [480,
    1200]) in one plan of shape 0, against the single-image calls, image by
    image: the single-image calls take shape 0 at these sizes too, so every
    image's levels, detector response, k and keypoints are bitwise equal."""
    K = gpu_lib
    sizes = batch_sizes(64, 3, 640, 1920, 480, 1200)
    seeds = [3000 + j for j in range(64)]
    note(f"[batch] full uneven workload, {len(sizes)} images, "
         f"{sum(w * h for w, h in sizes) / 1e6:.1f} Mpx")
    kb, imgs = make_batch(K, sizes, seeds, 0)
    kb.run()
    torch.cuda.synchronize()
    n_kp = 0
    for j, im in enumerate(imgs):
        ref = single(K, im)
        assert float(kb.k[j].item()) == float(ref.k.item()), j
        assert torch.equal(kb.levels[j], ref.levels), j
        assert torch.equal(kb.det[j], ref.det), j
        kp = kb.keypoints(j)
        assert np.array_equal(kp, ref.keypoints()), j
        n_kp += len(kp)
        del ref
    note(f"  64/64 images bitwise equal, {n_kp} keypoints")
    kb.close()


def test_detector_fork_threshold(gpu_lib):
    """The detector runs beside the steps from 32 Mpx per batch and after
    them below (8 x 1920x1200, 18.4 Mpx, measured faster that way); a batch
    without a detector has no detector levels in its segment."""
    K = gpu_lib
    below = K.KazeBatch([(1920, 1200)] * 8, shape=0)
    assert below.det_levels_in_segment == 0
    below.close()
    above = K.KazeBatch([(1920, 1200)] * 14, shape=0)  # 32.3 Mpx
    assert above.det_levels_in_segment == above.N
    above.close()
    nodet = K.KazeBatch([(1920, 1200)] * 14, shape=0, with_detector=False)
    assert nodet.det_levels_in_segment == 0
    nodet.close()


def test_large_batch_forks_detector_and_matches_eager(gpu_lib):
    """Above the size where the detector response runs beside the steps (a
    second stream inside the captured graph), replays still equal the eager
    sequence bitwise."""
    K = gpu_lib
    sizes = [(1920, 1200)] * 11 + [(1900, 1150), (1800, 1100), (1700, 1000), (1600, 1200)]
    note("[batch] large batch of %d images, %.1f Mpx" % (len(sizes), sum(w * h for w, h in sizes) / 1e6))
    kb, _ = make_batch(K, sizes, range(80, 80 + len(sizes)), 1)
    assert kb.det_levels_in_segment == kb.N
    kb.run(eager=True)
    torch.cuda.synchronize()
    ref_lv = [t.clone() for t in kb.levels]
    ref_det = [t.clone() for t in kb.det]
    ref_cnt = [int(c.item()) for c in kb.count]
    for r in range(2):
        for t in kb.det:
            t.fill_(-1.0)
        kb.run()
        torch.cuda.synchronize()
        for j in range(len(sizes)):
            assert torch.equal(kb.levels[j], ref_lv[j]), (r, j)
            assert torch.equal(kb.det[j], ref_det[j]), (r, j)
            assert int(kb.count[j].item()) == ref_cnt[j], (r, j)
    kb.close()


@pytest.mark.parametrize("window", ["3x3", "sigma"])
def test_batch_extrema_with_every_mask_bit_set(gpu_lib, window):
    """The batch's extrema kernel reads det only where the detector's mask
    bit (det above the threshold) is set; the single-image calls read every
    det value.  A threshold below every response sets every bit, so the
    mask kernel tests every position: its keypoints equal the scanning
    kernel's on ragged widths (partial mask words) and on both windows."""
    K = gpu_lib
    sizes = [(67, 45), (130, 97), (9, 13), (64, 64), (200, 33)]
    win = K.KAZE_WINDOW_3X3 if window == "3x3" else K.KAZE_WINDOW_SIGMA
    p = K.kaze_default_params(det_threshold=-1e30, extrema_window=win)
    cap = 1 << 16
    kb = K.KazeBatch(sizes, params=p, capacity=cap, shape=0)
    imgs = [kaze_image(W, H, 90 + j) for j, (W, H) in enumerate(sizes)]
    for x, im in zip(kb.inputs, imgs):
        x.copy_(torch.from_numpy(im))
    kb.run()
    torch.cuda.synchronize()
    for j, (im, (W, H)) in enumerate(zip(imgs, sizes)):
        kz = K.Kaze(W, H, p, capacity=cap)
        kz.run(torch.from_numpy(im).cuda())
        torch.cuda.synchronize()
        n = int(kb.count[j].item())
        note(f"[batch] every mask bit set, {window}, {W}x{H}: {n} extrema")
        assert 0 < n <= cap
        assert torch.equal(kb.det[j], kz.det)
        assert np.array_equal(kb.keypoints(j), kz.keypoints())
    kb.close()


@pytest.mark.parametrize("window", ["3x3", "sigma"])
def test_batch_extrema_at_extreme_shapes(gpu_lib, window):
    """The batch's masked extrema against the single-image calls' scan at
    the widest rows (4096 px: 64 mask words per row) and the thinnest
    images the library accepts, at the default threshold and at one that
    sets most bits."""
    K = gpu_lib
    sizes = [(4096, 9), (4000, 20), (64, 2100), (8, 8), (130, 1100)]
    win = K.KAZE_WINDOW_3X3 if window == "3x3" else K.KAZE_WINDOW_SIGMA
    imgs = [kaze_image(W, H, 110 + j) for j, (W, H) in enumerate(sizes)]
    for thr in (0.001, -1e30):
        p = K.kaze_default_params(det_threshold=thr, extrema_window=win)
        cap = 1 << 18
        kb = K.KazeBatch(sizes, params=p, capacity=cap, shape=0)
        for x, im in zip(kb.inputs, imgs):
            x.copy_(torch.from_numpy(im))
        kb.run()
        torch.cuda.synchronize()
        for j, (im, (W, H)) in enumerate(zip(imgs, sizes)):
            kz = K.Kaze(W, H, p, capacity=cap)
            kz.run(torch.from_numpy(im).cuda())
            torch.cuda.synchronize()
            n = int(kb.count[j].item())
            note(f"[batch] extreme shape {W}x{H}, {window}, threshold {thr:g}: {n} extrema")
            assert n <= cap
            assert np.array_equal(kb.keypoints(j), kz.keypoints())
        kb.close()
