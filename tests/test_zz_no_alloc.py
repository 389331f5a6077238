"""kaze_build_scale_space_noalloc (device-resident scratch) against
kaze_build_scale_space (caller workspace), through the C ABI: the same
kernels on the same scratch layout, so the levels and k must be bitwise
equal.  Two calls in a row on the shared scratch, the second smaller, and a
third at the first size again, so stale contents of a larger call cannot
leak into a smaller one or back."""
import numpy as np
import pytest
import torch

from synthetic import kaze_image

pytestmark = pytest.mark.gpu


def _pair(K, W, H, seed, **params):
    p = K.kaze_default_params(**params)
    N = K.kaze_num_levels(p)
    img = torch.from_numpy(kaze_image(W, H, seed)).cuda()
    ref_lev = torch.empty((N, H, W), dtype=torch.float32, device="cuda")
    ref_k = torch.empty(1, dtype=torch.float32, device="cuda")
    nb = K.kaze_workspace_bytes(W, H, p)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    K.kaze_build_scale_space(img, W, H, W, p, ref_lev, ref_k, ws, nb)
    lev = torch.full((N, H, W), float("nan"), dtype=torch.float32, device="cuda")
    k = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    K.kaze_build_scale_space_noalloc(img, W, H, W, p, lev, k)
    torch.cuda.synchronize()
    return ref_lev.cpu().numpy(), ref_k.item(), lev.cpu().numpy(), k.item()


def test_noalloc_equals_workspace_path(gpu_lib):
    K = gpu_lib
    for (W, H, seed) in [(1920, 1200, 2), (640, 480, 7), (1920, 1200, 3)]:
        print("noalloc %dx%d seed %d" % (W, H, seed), flush=True)
        ref, kr, out, k = _pair(K, W, H, seed)
        assert k == kr, (W, H, k, kr)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (W, H)


def test_noalloc_fed_and_substeps(gpu_lib):
    K = gpu_lib
    for params in (dict(scheme=K.KAZE_FED), dict(substeps=2)):
        print("noalloc 800x600", params, flush=True)
        ref, kr, out, k = _pair(K, 800, 600, 21, **params)
        assert k == kr
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), params


def test_noalloc_rejects_oversize(gpu_lib):
    K = gpu_lib
    p = K.kaze_default_params()
    img = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
    lev = torch.empty((1,), dtype=torch.float32, device="cuda")
    with pytest.raises(K.KazeError) as e:
        K.kaze_build_scale_space_noalloc(img, 4096, 4096, 4096, p, lev, lev)
    assert e.value.status == K.KAZE_ERR_UNSUPPORTED
