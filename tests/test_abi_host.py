"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, lays out its structs like a C compiler does, and validates arguments
before touching the GPU.  No kernel is launched here."""
import ctypes
import os
import re
import subprocess
import textwrap

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kaze.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("kaze.h", "kaze_surrogate.h")]


def _gpu_visible():
    import torch
    return torch.cuda.device_count() > 0


# These tests hand fake device addresses to entry points that must reject
# them before any launch; they only run where no kernel could execute.
no_gpu_only = pytest.mark.skipif(_gpu_visible(), reason="fake-pointer tests run without a GPU")


@pytest.fixture(scope="module")
def K():
    from paper_1706_06750_amd import build as B
    if not os.path.exists(B.LIB_PATH):
        B.build()
    from paper_1706_06750_amd import kaze
    return kaze


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*[\w\s\*]+?\b(kaze_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(K):
    from paper_1706_06750_amd import surrogate as S
    names = declared_functions()
    assert len(names) >= 23
    assert sorted(K.EXPORTS + S.EXPORTS) == names
    lib = ctypes.CDLL(K.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_c_compiler(K, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(textwrap.dedent("""
        #include <stdio.h>
        #include <stddef.h>
        #include "kaze.h"
        int main(void) {
          printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(kaze_params),
                 offsetof(kaze_params, octaves), offsetof(kaze_params, sublevels),
                 offsetof(kaze_params, sigma0), offsetof(kaze_params, sigma_cond),
                 offsetof(kaze_params, diffusivity), offsetof(kaze_params, k_bins),
                 offsetof(kaze_params, k_percentile), offsetof(kaze_params, k_override),
                 offsetof(kaze_params, det_threshold), sizeof(kaze_keypoint));
          return 0;
        }"""))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog),
                    "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    P = K.kaze_params
    want = [ctypes.sizeof(P)] + [getattr(P, f).offset for f in
                                 ("octaves", "sublevels", "sigma0", "sigma_cond", "diffusivity",
                                  "k_bins", "k_percentile", "k_override", "det_threshold")]
    want.append(ctypes.sizeof(K.kaze_keypoint))
    assert got == want
    prog2 = tmp_path / "layout2.c"
    prog2.write_text(textwrap.dedent("""
        #include <stdio.h>
        #include <stddef.h>
        #include "kaze.h"
        int main(void) {
          printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(kaze_image_desc),
                 offsetof(kaze_image_desc, img), offsetof(kaze_image_desc, W),
                 offsetof(kaze_image_desc, H), offsetof(kaze_image_desc, ld_img),
                 offsetof(kaze_image_desc, levels), offsetof(kaze_image_desc, det),
                 offsetof(kaze_image_desc, k), offsetof(kaze_image_desc, kps),
                 offsetof(kaze_image_desc, capacity), offsetof(kaze_image_desc, count),
                 sizeof(kaze_batch_config));
          return 0;
        }"""))
    exe2 = tmp_path / "layout2"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog2),
                    "-o", str(exe2)], check=True)
    got2 = [int(v) for v in subprocess.run([str(exe2)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    D = K.kaze_image_desc
    want2 = [ctypes.sizeof(D)] + [getattr(D, f).offset for f in
                                  ("img", "W", "H", "ld_img", "levels", "det", "k", "kps",
                                   "capacity", "count")] + [ctypes.sizeof(K.kaze_batch_config)]
    assert got2 == want2


def test_defaults_and_schedule_match_oracle(K):
    p = K.kaze_default_params()
    assert (p.octaves, p.sublevels, p.k_bins, p.diffusivity) == (4, 4, 300, K.KAZE_G2)
    assert (p.sigma0, p.sigma_cond, p.k_percentile, p.det_threshold) == (1.6, 1.0, 0.7, 0.001)
    assert (p.scheme, p.extrema_window) == (K.KAZE_AOS, K.KAZE_WINDOW_3X3)
    sch = K.kaze_schedule(p)
    ref = O.level_schedule(1.6, 4, 4)
    assert len(sch) == len(ref) == K.kaze_num_levels(p)
    for i, (a, b) in enumerate(zip(sch, ref)):
        assert a["sigma"] == pytest.approx(b["sigma"], rel=1e-15)
        assert a["t"] == pytest.approx(b["t"], rel=1e-15)
        if i:
            assert a["tau"] == pytest.approx(b["t"] - ref[i - 1]["t"], rel=1e-14)
        sn = b["sigma"] / 2 ** b["o"]
        assert a["sigma_norm"] == pytest.approx(sn, rel=1e-15)
        assert a["deriv_step"] == O.derivative_step(sn)


def test_workspace_bytes(K):
    p = K.kaze_default_params()
    w = K.kaze_workspace_bytes(1920, 1200, p)
    assert w >= 1920 * 1200 * 4 and w % 256 == 0
    assert K.kaze_workspace_bytes(7, 100, p) == 0
    assert K.kaze_workspace_bytes(100, 5000, p) == 0
    assert K.kaze_workspace_bytes(4097, 64, p) == 0
    assert K.kaze_workspace_bytes(4096, 4096, p) > 0
    assert K.kaze_workspace_bytes(64, 64, K.kaze_default_params(sigma_cond=1.4)) == 0
    bad = K.kaze_default_params(octaves=0)
    assert K.kaze_workspace_bytes(64, 64, bad) == 0


@pytest.mark.parametrize("field,value,status", [
    ("octaves", 0, -1), ("sublevels", 0, -1), ("octaves", 17, -4), ("sigma0", 0.0, -1),
    ("sigma0", 6.0, -4), ("diffusivity", 3, -1), ("k_percentile", 0.0, -1),
    ("k_percentile", 1.5, -1), ("k_bins", 0, -1), ("k_bins", 5000, -1),
    ("sigma_cond", 1.4, -4), ("scheme", 2, -1), ("extrema_window", 2, -1),
    ("extrema_window", -1, -1), ("substeps", 0, -1), ("substeps", 65, -1),
])
@no_gpu_only
def test_invalid_params_rejected_before_launch(K, field, value, status):
    p = K.kaze_default_params(**{field: value})
    with pytest.raises(K.KazeError) as e:
        K.kaze_build_scale_space(16, 64, 64, 64, p, 16, 16, 256, 1 << 30, 0)
    assert e.value.status == status


@no_gpu_only
def test_invalid_buffers_rejected_before_launch(K):
    p = K.kaze_default_params()
    ws = K.kaze_workspace_bytes(64, 64, p)
    cases = [
        dict(img=0), dict(levels=0), dict(k_out=0), dict(W=7), dict(H=5000),
        dict(ld=63), dict(ws=0), dict(ws=128 + 256), dict(ws_bytes=ws - 1), dict(img=18),
    ]
    for c in cases:
        a = dict(img=256, W=64, H=64, ld=64, levels=512, k_out=1024, ws=4096, ws_bytes=ws)
        a.update(c)
        with pytest.raises(K.KazeError) as e:
            K.kaze_build_scale_space(a["img"], a["W"], a["H"], a["ld"], p, a["levels"],
                                     a["k_out"], a["ws"], a["ws_bytes"], 0)
        assert e.value.status in (-1, -2, -4), c
    with pytest.raises(K.KazeError):
        K.kaze_find_extrema(256, 64, 64, p, 0, 5, 512, 0)       # capacity without buffer
    with pytest.raises(K.KazeError):
        K.kaze_find_extrema(256, 64, 64, p, 0, -1, 512, 0)
    with pytest.raises(K.KazeError):
        K.kaze_detector_response(0, 64, 64, p, 512, 0)
    with pytest.raises(K.KazeError):
        K.kaze_aos_step(256, 512, 64, 64, 0.0, 1024, 4096, ws, 0)  # tau must be > 0
    with pytest.raises(K.KazeError):
        K.kaze_conductivity(256, 64, 64, p, -1.0, 512, 0)
    with pytest.raises(K.KazeError):
        K.kaze_copy_f32(8, 1024, 16, 0)                         # misaligned
    with pytest.raises(K.KazeError):
        K.kaze_profile_begin("no_such_kernel")


def test_kernel_names(K):
    names = K.kaze_kernel_names()
    for n in ("aos_reduce", "aos_iface", "aos_recover", "cond", "det", "nms"):
        assert n in names


def test_batch_workspace_query(K):
    p = K.kaze_default_params()
    D = K.kaze_image_desc
    small = [D(256, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192),
             D(256, 300, 200, 300, 512, 1024, 2048, 4096, 10, 8192)]
    sizes = [K.kaze_batch_workspace_bytes(small, p, s) for s in range(len(K.AOS_SHAPES))]
    assert all(v > 0 and v % 256 == 0 for v in sizes)
    assert K.kaze_batch_workspace_bytes(small, p) == max(sizes)
    # every shape fits every accepted size; 4096 is the largest side
    tall = [D(256, 100, 4096, 100, 512, 1024, 2048, 4096, 10, 8192)]
    assert all(K.kaze_batch_workspace_bytes(tall, p, s) > 0 for s in range(len(K.AOS_SHAPES)))
    assert K.kaze_batch_workspace_bytes([D(256, 100, 4097, 100, 512, 0, 2048, 0, 0, 0)], p) == 0
    assert K.kaze_batch_workspace_bytes(small, p, len(K.AOS_SHAPES)) == 0
    assert K.kaze_batch_workspace_bytes([D(256, 7, 80, 7, 512, 0, 2048, 0, 0, 0)], p) == 0


def test_aos_shape_table(K):
    """The library's shape table is the one include/kaze.h documents."""
    hdr = open(HEADER).read()
    rows = re.findall(r"^ \*\s+(\d)\s+(\d+)x(\d+)\s+(\d+)\s+(\d+)\s+(\d+)\s+(\d)\s*$", hdr,
                      flags=re.M)
    m = re.search(r"#define KAZE_AOS_SHAPES (\d+)", hdr)
    assert m and int(m.group(1)) == len(K.AOS_SHAPES) == len(rows)
    for r in rows:
        a = K.AOS_SHAPES[int(r[0])]
        assert (a["tile_w"], a["tile_h"], a["row_chunk"], a["col_chunk"], a["iface_m"],
                a["chunk_lanes"]) == tuple(int(v) for v in r[1:]), r
        # whole chunks per tile: the kernels' lane mapping assumes it
        assert a["tile_w"] % a["row_chunk"] == 0 and a["tile_h"] % a["col_chunk"] == 0
    for bad in (-1, len(K.AOS_SHAPES)):
        assert K.lib.kaze_aos_shape_info(bad, None, None, None, None, None, None) == \
            K.KAZE_ERR_INVALID_ARG


def test_batch_workspace_holds_detector_masks(K):
    """A batch that finds extrema (count given) needs, per image, N planes of
    H rows of 64-bit threshold-mask words (a 256-byte aligned region) more
    than one that stops at det: one word per detector strip at the largest
    Scharr step (8: strips of 64 - 16 = 48 columns)."""
    p = K.kaze_default_params()
    N = K.kaze_num_levels(p)
    D = K.kaze_image_desc
    dims = [(100, 80), (300, 200), (64, 9)]
    with_nms = [D(256, W, H, W, 512, 1024, 2048, 4096, 10, 8192) for W, H in dims]
    det_only = [D(256, W, H, W, 512, 1024, 2048, 0, 0, 0) for W, H in dims]
    words = lambda W: 1 if W <= 48 else (W + 47) // 48
    masks = sum((N * H * words(W) * 8 + 255) // 256 * 256 for W, H in dims)
    for s in range(len(K.AOS_SHAPES)):
        a = K.kaze_batch_workspace_bytes(with_nms, p, s)
        b = K.kaze_batch_workspace_bytes(det_only, p, s)
        assert a > 0 and b > 0 and a - b == masks


@no_gpu_only
def test_batch_create_rejects_before_any_device_call(K):
    p = K.kaze_default_params()
    D = K.kaze_image_desc
    good = D(256, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192)
    ws = K.kaze_batch_workspace_bytes([good], p, 0)
    cases = [
        [D(0, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192)],        # no input
        [D(256, 100, 80, 90, 512, 1024, 2048, 4096, 10, 8192)],       # ld < W
        [good, D(256, 100, 80, 100, 512, 0, 2048, 4096, 10, 8192)],   # det for some only
        [D(256, 100, 80, 100, 512, 1024, 2048, 0, 10, 8192)],         # capacity without kps
        [D(258, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192)],      # misaligned input
    ]
    for c in cases:
        with pytest.raises(K.KazeError):
            K.kaze_batch_create(c, p, 0, 1 << 20, ws)
    with pytest.raises(K.KazeError):
        K.kaze_batch_create([good], p, 0, 1 << 20, ws - 1)            # workspace too small
    with pytest.raises(K.KazeError):
        K.kaze_batch_create([good], p, 7, 1 << 20, ws)                # no such shape


def test_surrogate_sizes_and_rejections(K):
    from oracle import cnn_oracle as C
    from paper_1706_06750_amd import surrogate as S
    assert S.kaze_sg_param_count() == C.param_count() == 38177
    assert S.kaze_sg_packed_bytes() % 256 == 0 and S.kaze_sg_packed_bytes() > 38177 * 2
    assert S.kaze_sg_workspace_bytes(0, 64, 64, 0) == 0
    assert S.kaze_sg_workspace_bytes(1, 8193, 64, 0) == 0
    assert S.kaze_sg_workspace_bytes(1, 64, 64, 2) == 0
    inf = S.kaze_sg_workspace_bytes(2, 100, 37, 0)
    tr = S.kaze_sg_workspace_bytes(2, 100, 37, 1)
    # inference holds the input planes and two activation buffers
    assert inf >= 2 * 102 * 39 * (8 + 2 * 32) * 2 and tr > 4 * inf
    with pytest.raises(K.KazeError) as e:
        S.kaze_sg_plan_create(1, 64, 64, 0, None, 1 << 20, stream=0)
    assert e.value.status == K.KAZE_ERR_WORKSPACE
    with pytest.raises(K.KazeError):
        S.kaze_sg_plan_create(1, 0, 64, 0, None, 1 << 20, stream=0)
    with pytest.raises(K.KazeError):
        S.kaze_sg_adam(None, None, None, None, 10, 1, stream=0)
    with pytest.raises(K.KazeError):
        S.kaze_sg_pack(None, None, stream=0)


@no_gpu_only
def test_surrogate_rejects_before_launch(K):
    from paper_1706_06750_amd import surrogate as S
    fake = 1 << 40
    with pytest.raises(K.KazeError) as e:   # too small
        S.kaze_sg_plan_create(1, 64, 64, 1, fake, 1024, stream=0)
    assert e.value.status == K.KAZE_ERR_WORKSPACE
    with pytest.raises(K.KazeError) as e:   # misaligned
        S.kaze_sg_plan_create(1, 64, 64, 0, fake + 8, 1 << 30, stream=0)
    assert e.value.status == K.KAZE_ERR_WORKSPACE
    with pytest.raises(K.KazeError):        # misaligned packed weights
        S.kaze_sg_pack(fake, fake + 4, stream=0)
    with pytest.raises(K.KazeError):        # bad Adam hyper-parameters
        S.kaze_sg_adam(fake, fake, fake, fake, 10, 1, lr=-1.0, stream=0)


def test_fed_scheme_is_single_image_only(K):
    p = K.kaze_default_params()
    assert p.scheme == K.KAZE_AOS
    p.scheme = K.KAZE_FED
    D = K.kaze_image_desc
    small = [D(256, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192)]
    assert K.kaze_batch_workspace_bytes(small, p) == 0
    q = K.kaze_default_params()
    fed_ws = K.kaze_workspace_bytes(100, 80, p)
    aos_ws = K.kaze_workspace_bytes(100, 80, q)
    assert fed_ws >= aos_ws + 100 * 80 * 4   # the second plane of the explicit steps
    p.scheme = 7
    assert K.kaze_workspace_bytes(100, 80, p) == 0



@no_gpu_only
def test_refine_arguments_rejected_before_launch(K):
    p = K.kaze_default_params()
    ok = dict(det=256, W=64, H=64, kps=512, count=768, capacity=4, r=10.0, out=1024)
    cases = [dict(capacity=-1), dict(r=1.0), dict(r=0.5), dict(r=float("inf")), dict(det=0),
             dict(kps=0), dict(count=0), dict(out=0), dict(out=1026), dict(W=7), dict(H=4097)]
    for c in cases:
        a = dict(ok, **c)
        with pytest.raises(K.KazeError):
            K.kaze_refine_keypoints(a["det"], a["W"], a["H"], p, a["kps"], a["count"],
                                    a["capacity"], a["r"], a["out"], 0)
    bad = K.kaze_default_params(octaves=0)
    with pytest.raises(K.KazeError):
        K.kaze_refine_keypoints(256, 64, 64, bad, 512, 768, 4, 10.0, 1024, 0)


def test_substeps_parameter(K):
    p = K.kaze_default_params()
    assert p.substeps == 1
    base = K.kaze_workspace_bytes(320, 240, p)
    p2 = K.kaze_default_params(substeps=3)
    assert K.kaze_workspace_bytes(320, 240, p2) == base + 320 * 240 * 4
    for bad in (0, 65, -2):
        assert K.kaze_workspace_bytes(320, 240, K.kaze_default_params(substeps=bad)) == 0
    D = K.kaze_image_desc
    im = [D(256, 100, 80, 100, 512, 1024, 2048, 4096, 10, 8192)]
    assert K.kaze_batch_workspace_bytes(im, p2, 0) > K.kaze_batch_workspace_bytes(im, p, 0)


def test_surrogate_rejects_substeps(K):
    from paper_1706_06750_amd import surrogate as S
    c = S.kaze_sg_default_config()
    assert S.kaze_sg_scale_space_workspace_bytes(64, 64, K.kaze_default_params(), c) > 0
    assert S.kaze_sg_scale_space_workspace_bytes(64, 64, K.kaze_default_params(substeps=2), c) == 0


@no_gpu_only
def test_describe_arguments_rejected_before_launch(K):
    p = K.kaze_default_params()
    ok = dict(lx=256, ly=512, W=64, H=64, kps=768, count=1024, capacity=4, ang=1280, desc=1536)
    for c in (dict(capacity=-1), dict(lx=0), dict(ly=0), dict(kps=0), dict(count=0),
              dict(ang=0), dict(desc=0), dict(desc=1538), dict(W=7), dict(H=4097)):
        a = dict(ok, **c)
        with pytest.raises(K.KazeError):
            K.kaze_describe_keypoints(a["lx"], a["ly"], a["W"], a["H"], p, a["kps"], a["count"],
                                      a["capacity"], a["ang"], a["desc"], 0)
    for c in (dict(levels=0), dict(lx=0), dict(ly=0), dict(W=7)):
        a = dict(dict(levels=256, lx=512, ly=768, W=64), **c)
        with pytest.raises(K.KazeError):
            K.kaze_derivatives(a["levels"], a["W"], 64, p, a["lx"], a["ly"], 0)


def test_noalloc_scratch_limit(K):
    p = K.kaze_default_params()
    assert K.kaze_workspace_bytes(3840, 2160, p) <= K.KAZE_NOALLOC_SCRATCH_BYTES
    assert K.kaze_workspace_bytes(4096, 4096, p) > K.KAZE_NOALLOC_SCRATCH_BYTES
    fed = K.kaze_default_params(scheme=K.KAZE_FED)
    assert K.kaze_workspace_bytes(2560, 1600, fed) <= K.KAZE_NOALLOC_SCRATCH_BYTES
    hdr = open(HEADER).read()
    m = re.search(r"#define KAZE_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == K.KAZE_NOALLOC_SCRATCH_BYTES


@no_gpu_only
def test_noalloc_rejects_before_any_device_call(K):
    p = K.kaze_default_params()
    cases = [
        (dict(W=4096, H=4096), -4),           # scratch would exceed the static array
        (dict(img=0), -1), (dict(levels=0), -1), (dict(k_out=0), -1), (dict(W=7), -1),
        (dict(ld=63), -1), (dict(img=18), -1), (dict(H=5000), -4),
    ]
    for c, status in cases:
        a = dict(img=256, W=64, H=64, ld=None, levels=512, k_out=1024)
        a.update(c)
        ld = a["ld"] if a["ld"] is not None else a["W"]
        with pytest.raises(K.KazeError) as e:
            K.kaze_build_scale_space_noalloc(a["img"], a["W"], a["H"], ld, p, a["levels"],
                                             a["k_out"], 0)
        assert e.value.status == status, c
    bad = K.kaze_default_params(octaves=0)
    with pytest.raises(K.KazeError) as e:
        K.kaze_build_scale_space_noalloc(256, 64, 64, 64, bad, 512, 1024, 0)
    assert e.value.status == -1
