"""Pitched inputs (row pitch ld_img > W) through the C ABI: the single-image
call and a batch read the image rows at the given pitch and produce exactly
what the same image gives densely packed, and the oracle's levels."""
import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image
from kaze_parity import LEVEL_TOL, compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("W,H,ld", [(333, 250, 400), (320, 240, 321), (61, 47, 64)])
def test_single_image_pitched_input(gpu_lib, W, H, ld):
    K = gpu_lib
    img = kaze_image(W, H, 77)
    note(f"[pitched] {W}x{H} ld {ld}")
    buf = torch.full((H, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :W] = torch.from_numpy(img).cuda()
    view = buf[:, :W]
    assert view.stride(0) == ld
    kp = K.Kaze(W, H)
    kp.run(view)
    kd = K.Kaze(W, H)
    kd.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    assert torch.equal(kp.levels, kd.levels)
    assert torch.equal(kp.det, kd.det)
    assert kp.k.item() == kd.k.item()
    lev_o, k_o = O.build_scale_space(img.astype(np.float64))
    det_o = O.detector_response(lev_o)
    err = float(np.max(np.abs(kp.levels.cpu().numpy() - lev_o)))
    common, bad_g, bad_o = compare_keypoints(kp.keypoints(), O.find_extrema(det_o, 0.001),
                                             det_o, 0.001)
    note(f"  worst level err {err:.2e}, keypoints common {common}")
    assert err <= LEVEL_TOL
    assert not bad_g and not bad_o


def test_batch_pitched_inputs(gpu_lib):
    K = gpu_lib
    sizes = [(67, 45), (320, 240), (130, 260), (9, 13)]
    note(f"[pitched] batch {sizes} pad 37")
    imgs = [kaze_image(W, H, 90 + j) for j, (W, H) in enumerate(sizes)]
    kb = K.KazeBatch(sizes, shape=0, ld_pad=37)
    kd = K.KazeBatch(sizes, shape=0)
    for j, im in enumerate(imgs):
        assert kb.inputs[j].stride(0) == sizes[j][0] + 37
        kb.inputs[j].copy_(torch.from_numpy(im))
        kd.inputs[j].copy_(torch.from_numpy(im))
    kb.run()
    kd.run()
    torch.cuda.synchronize()
    for j in range(len(sizes)):
        assert torch.equal(kb.levels[j], kd.levels[j]), j
        assert torch.equal(kb.det[j], kd.det[j]), j
        assert np.array_equal(kb.keypoints(j), kd.keypoints(j)), j
    kb.close()
    kd.close()
