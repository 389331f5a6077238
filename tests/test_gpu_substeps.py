"""Sub-steps per level on the GPU against the FP64 oracle, through the C ABI:
params.substeps = m splits every level step into m equal AOS steps (or FED
cycles), each with the conductivity of its own starting image.  The bar is
the plain path's: 1e-4 per level on [0, 1] images and the keypoint rule;
the batched form equals the single-image path bitwise."""
import numpy as np
import pytest

import oracle as O
from synthetic import kaze_image
from kaze_parity import LEVEL_TOL, compare_keypoints, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def run(K, img, **kw):
    H, W = img.shape
    p = K.kaze_default_params(**kw)
    kz = K.Kaze(W, H, p)
    kz.run(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    return kz


@pytest.mark.parametrize("W,H,seed,m,scheme", [(160, 120, 1, 2, "aos"), (67, 45, 5, 3, "aos"),
                                               (130, 97, 6, 4, "aos"), (120, 90, 2, 2, "fed")])
def test_substeps_vs_oracle(gpu_lib, W, H, seed, m, scheme):
    K = gpu_lib
    img = kaze_image(W, H, seed)
    kz = run(K, img, substeps=m, scheme=K.KAZE_AOS if scheme == "aos" else K.KAZE_FED)
    lev_o, k_o = O.build_scale_space(img.astype(np.float64), scheme=scheme, substeps=m)
    det_o = O.detector_response(lev_o)
    kp_o = O.find_extrema(det_o, 0.001)
    lev_g = kz.levels.cpu().numpy()
    errs = [float(np.abs(lev_g[i] - lev_o[i]).max()) for i in range(len(lev_o))]
    note(f"[substeps] {W}x{H} seed {seed} m {m} {scheme}: max|L - L_orc| per level "
         + " ".join("%.1e" % e for e in errs))
    assert float(kz.k.item()) == pytest.approx(k_o, rel=1e-4)
    assert max(errs) <= LEVEL_TOL
    common, bad_g, bad_o = compare_keypoints(kz.keypoints(), kp_o, det_o, 0.001)
    note(f"  keypoints {common} common, unexcused {len(bad_g)} + {len(bad_o)}")
    assert not bad_g and not bad_o


def test_one_substep_is_the_default_path(gpu_lib):
    K = gpu_lib
    img = kaze_image(96, 80, 3)
    a = run(K, img)
    b = run(K, img, substeps=1)
    c = run(K, img, substeps=2)
    assert torch.equal(a.levels, b.levels)
    assert torch.equal(a.levels[0], c.levels[0]) and not torch.equal(a.levels[1:], c.levels[1:])


@pytest.mark.parametrize("shape", [0, 2])
def test_substeps_batch_equals_single(gpu_lib, shape):
    """Sub-steps in a batch plan against the single-image calls (shape 0 at
    these sizes): bitwise for shape 0; shape 2 (60x64 tiles, one lane per
    chunk) rounds differently, so within 1e-5 with the keypoint sets equal up
    to the excuse rule."""
    K = gpu_lib
    keys = ("row_chunk", "col_chunk", "iface_m", "chunk_lanes")
    exact = all(K.AOS_SHAPES[shape][k] == K.AOS_SHAPES[0][k] for k in keys)
    p = K.kaze_default_params(substeps=3)
    sizes = [(160, 120), (67, 45), (31, 33)]
    kb = K.KazeBatch(sizes, params=p, shape=shape)
    imgs = [kaze_image(W, H, 70 + j) for j, (W, H) in enumerate(sizes)]
    for x, im in zip(kb.inputs, imgs):
        x.copy_(torch.from_numpy(im))
    kb.run()
    torch.cuda.synchronize()
    for j, im in enumerate(imgs):
        ref = run(K, im, substeps=3)
        if exact:
            assert torch.equal(kb.levels[j], ref.levels)
            assert np.array_equal(kb.keypoints(j), ref.keypoints())
        else:
            assert (kb.levels[j] - ref.levels).abs().max().item() <= 1e-5
            det_ref = ref.det.cpu().numpy().astype(np.float64)
            _, bad_b, bad_r = compare_keypoints(kb.keypoints(j), ref.keypoints(), det_ref, 0.001)
            assert not bad_b and not bad_r, (j, bad_b, bad_r)
    kb.close()

