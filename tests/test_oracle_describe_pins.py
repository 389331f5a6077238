"""Pins of the oracle's description stage (Sec. II-C, Sec. III-C): exact
derivatives of linear ramps, bilinear sampling and its mirror symmetry,
the orientation of uniform fields, a brute-force sweep of the sliding
sector, equivariance under a quarter turn, and closed forms of the
descriptor for uniform and half-plane fields."""
import math

import numpy as np
import pytest

import oracle as O


def test_first_derivatives_of_a_ramp():
    H, W = 40, 50
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    lev = np.stack([0.003 * xx - 0.002 * yy + 0.5] * 16)
    lx, ly = O.first_derivatives(lev)
    for s in O.level_schedule():
        i, sn = s["i"], s["sigma"] / 2 ** s["o"]
        st = O.derivative_step(sn)
        core = (slice(st, H - st), slice(st, W - st))
        assert np.allclose(lx[i][core], sn * 0.003, atol=1e-15, rtol=1e-12)
        assert np.allclose(ly[i][core], -sn * 0.002, atol=1e-15, rtol=1e-12)


def test_bilinear_exact_and_mirrored():
    rng = np.random.default_rng(1)
    H, W = 7, 9
    img = rng.random((H, W))
    yy, xx = np.mgrid[0:H, 0:W]
    assert np.array_equal(O.bilinear(img, xx.astype(float), yy.astype(float)), img)
    lin = 0.3 * xx + 0.7 * yy + 1.0
    x = rng.uniform(0, W - 1, 200)
    y = rng.uniform(0, H - 1, 200)
    assert np.allclose(O.bilinear(lin, x, y), 0.3 * x + 0.7 * y + 1.0, atol=1e-12)
    # half-sample mirror about -0.5 and period 2n
    x = rng.uniform(-30, 30, 500)
    y = rng.uniform(-30, 30, 500)
    v = O.bilinear(img, x, y)
    assert np.allclose(v, O.bilinear(img, -1.0 - x, y), atol=1e-12)
    assert np.allclose(v, O.bilinear(img, x, -1.0 - y), atol=1e-12)
    assert np.allclose(v, O.bilinear(img, x + 2 * W, y - 2 * H), atol=1e-12)
    assert np.allclose(O.bilinear(img, -0.5, 3.0), img[3, 0])


@pytest.mark.parametrize("alpha", [0.3, -2.0, 3.1, math.pi / 2])
def test_uniform_field_orientation(alpha):
    lx = np.full((60, 60), math.cos(alpha))
    ly = np.full((60, 60), math.sin(alpha))
    t, _ = O.dominant_orientation(lx, ly, 30.0, 29.5, 2.3)
    assert abs(math.remainder(t - alpha, 2 * math.pi)) < 1e-12


def smooth_field(n, seed):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    return (gaussian_filter(rng.normal(size=(n, n)), 3.0, mode="reflect"),
            gaussian_filter(rng.normal(size=(n, n)), 3.0, mode="reflect"))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sector_sums_match_a_brute_force_sweep(seed):
    lx, ly = smooth_field(64, seed)
    x, y, s = 31.3, 30.6, 1.7
    _, lengths = O.dominant_orientation(lx, ly, x, y, s)
    uv = np.array(O.orientation_samples(), dtype=float)
    w = np.exp(-(uv ** 2).sum(1) / 12.5)
    rx = w * O.bilinear(lx, x + s * uv[:, 0], y + s * uv[:, 1])
    ry = w * O.bilinear(ly, x + s * uv[:, 0], y + s * uv[:, 1])
    phi = np.arctan2(ry, rx)
    best = 0.0
    for a in np.linspace(-math.pi, math.pi, 20001):
        m = np.mod(phi - a, 2 * math.pi) <= math.pi / 3
        best = max(best, math.hypot(rx[m].sum(), ry[m].sum()))
    assert best <= lengths.max() + 1e-12
    assert best > lengths.max() * (1 - 1e-6)


def quarter_turn(lx, ly):
    """Field turned by +90 degrees about the centre of a square image:
    position (x, y) -> (n-1-y, x), vector (a, b) -> (-b, a)."""
    n = lx.shape[0]
    lx2, ly2 = np.empty_like(lx), np.empty_like(ly)
    y, x = np.mgrid[0:n, 0:n]
    lx2[x, n - 1 - y] = -ly[y, x]
    ly2[x, n - 1 - y] = lx[y, x]
    return lx2, ly2


@pytest.mark.parametrize("seed", [3, 4])
def test_quarter_turn_equivariance(seed):
    n = 64
    lx, ly = smooth_field(n, seed)
    lx2, ly2 = quarter_turn(lx, ly)
    x, y, s = 30.0, 27.0, 2.0
    t1, _ = O.dominant_orientation(lx, ly, x, y, s)
    t2, _ = O.dominant_orientation(lx2, ly2, n - 1 - y, x, s)
    assert abs(math.remainder(t2 - t1 - math.pi / 2, 2 * math.pi)) < 1e-9
    d1 = O.msurf_descriptor(lx, ly, x, y, s, t1)
    d2 = O.msurf_descriptor(lx2, ly2, n - 1 - y, x, s, t2)
    assert np.allclose(d1, d2, atol=1e-9)


def gauss_sum_grid():
    t = np.arange(9) - 4.0
    return (np.exp(-t ** 2 / 12.5).sum()) ** 2


def test_descriptor_of_a_uniform_field():
    lx, ly = np.ones((80, 80)), np.zeros((80, 80))
    d = O.msurf_descriptor(lx, ly, 40.0, 40.0, 1.3, 0.0).reshape(4, 4, 4)
    w2 = np.array([[math.exp(-((a - 1.5) ** 2 + (b - 1.5) ** 2) / 4.5) for a in range(4)]
                   for b in range(4)])
    ref = np.zeros((4, 4, 4))
    ref[:, :, 0] = ref[:, :, 2] = w2 * gauss_sum_grid()
    ref /= np.linalg.norm(ref)
    assert np.allclose(d, ref, atol=1e-12)
    # turned by theta the field is seen at -theta: d_u = cos, d_v = -sin
    th = 0.4
    d = O.msurf_descriptor(lx, ly, 40.0, 40.0, 1.3, th).reshape(4, 4, 4)
    ref = np.zeros((4, 4, 4))
    g = w2 * gauss_sum_grid()
    ref[:, :, 0], ref[:, :, 1] = g * math.cos(th), -g * math.sin(th)
    ref[:, :, 2], ref[:, :, 3] = g * math.cos(th), g * math.sin(th)
    ref /= np.linalg.norm(ref)
    assert np.allclose(d, ref, atol=1e-12)


def test_descriptor_layout_and_invariances():
    # Lx = 1 right of the keypoint only: the subregions along +u (columns
    # a = 2, 3) carry it, a = 0 none
    lx = np.zeros((80, 80))
    lx[:, 41:] = 1.0
    d = O.msurf_descriptor(lx, np.zeros_like(lx), 40.0, 40.0, 1.0, 0.0).reshape(4, 4, 4)
    assert np.all(d[:, 0, :] == 0.0) and np.all(d[:, 3, 0] > 0) and np.all(d[:, :, 1] == 0)
    lx, ly = smooth_field(64, 5)
    d1 = O.msurf_descriptor(lx, ly, 31.0, 33.0, 1.6, 0.7)
    assert abs(np.linalg.norm(d1) - 1.0) < 1e-12
    assert np.allclose(O.msurf_descriptor(3 * lx, 3 * ly, 31.0, 33.0, 1.6, 0.7), d1, atol=1e-13)
    assert np.array_equal(O.msurf_descriptor(0 * lx, 0 * ly, 31.0, 33.0, 1.6, 0.7), np.zeros(64))


def test_describe_keypoints_uses_the_level_scale():
    lx, ly = smooth_field(64, 6)
    L = np.stack([lx] * 16)
    M = np.stack([ly] * 16)
    kps = np.array([[3, 30.5, 31.25, 0.0], [9, 28.0, 33.0, 0.0]])
    th, d = O.describe_keypoints(L, M, kps)
    sch = O.level_schedule()
    for j, (lev, y, x, _) in enumerate(kps):
        s = sch[int(lev)]["sigma"]
        t, _ = O.dominant_orientation(lx, ly, x, y, s)
        assert th[j] == t
        assert np.array_equal(d[j], O.msurf_descriptor(lx, ly, x, y, s, t))
