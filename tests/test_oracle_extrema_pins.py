"""Pins of the oracle's exact cross-level extrema (Sec. II-B, Sec. III-B,
Sec. IV): a brute-force loop over every pixel and window position, the
reduction to the 3x3x3 variant, the subset property the paper reports,
planted peaks at and beyond the window edge, clipping at the border and
ties."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def brute(det, thr, radii):
    N, H, W = det.shape
    out = set()
    for i in range(1, N - 1):
        h = radii[i]
        for y in range(1, H - 1):
            for x in range(1, W - 1):
                v = det[i, y, x]
                if not v > thr:
                    continue
                ok = True
                for yy in range(H):
                    for xx in range(W):
                        if abs(yy - y) <= 1 and abs(xx - x) <= 1 and (yy, xx) != (y, x):
                            ok = ok and v > det[i, yy, xx]
                        if abs(yy - y) <= h and abs(xx - x) <= h:
                            ok = ok and v > det[i - 1, yy, xx] and v > det[i + 1, yy, xx]
                if ok:
                    out.add((i, y, x))
    return out


def as_set(kps):
    return {tuple(int(v) for v in r[:3]) for r in kps}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_windowed_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    det = rng.normal(0, 1, size=(6, 11, 13))
    radii = [1, 1, 2, 3, 2, 1]
    got = O.find_extrema(det, 0.2, radii)
    assert as_set(got) == brute(det, 0.2, radii)
    assert len(got) > 0
    # responses are the det values at the positions
    for lev, y, x, v in got:
        assert v == det[int(lev), int(y), int(x)]


@pytest.mark.parametrize("seed", [3, 4])
def test_radius_one_is_the_3x3x3_variant(seed):
    rng = np.random.default_rng(seed)
    det = rng.normal(0, 1, size=(5, 30, 40))
    a = O.find_extrema(det, 0.0)
    b = O.find_extrema(det, 0.0, [1] * 5)
    assert np.array_equal(a, b) and len(a) > 10


def test_exact_set_is_a_subset_on_a_real_response():
    from synthetic import kaze_image
    img = kaze_image(96, 80, 2).astype(np.float64)
    lev, _ = O.build_scale_space(img)
    det = O.detector_response(lev)
    radii = [O.cross_level_radius(s["sigma"]) for s in O.level_schedule()]
    approx = as_set(O.find_extrema(det, 0.001))
    exact = as_set(O.find_extrema(det, 0.001, radii))
    assert exact <= approx and len(exact) > 0
    assert exact == brute(det, 0.001, radii)


@pytest.mark.parametrize("dist,h,kept", [(2, 1, True), (2, 2, False), (3, 2, True), (3, 3, False)])
def test_planted_peak_against_the_next_level(dist, h, kept):
    det = np.zeros((4, 21, 21))
    det[1, 10, 10] = 1.0
    det[2, 10, 10 + dist] = 1.5   # higher response directly beside, one level up
    got = as_set(O.find_extrema(det, 0.5, [1, h, 1, 1]))
    assert ((1, 10, 10) in got) == kept


def test_window_is_clipped_at_the_border():
    det = np.zeros((3, 9, 9))
    det[1, 1, 1] = 1.0
    det[0, 0, 0] = 0.9          # inside the clipped window, lower: kept
    got = as_set(O.find_extrema(det, 0.5, [1, 4, 1]))
    assert got == {(1, 1, 1)}
    det[2, 5, 5] = 1.0          # equal, at distance 4: rejected (strict)
    assert as_set(O.find_extrema(det, 0.5, [1, 4, 1])) == set()
    assert as_set(O.find_extrema(det, 0.5, [1, 3, 1])) == {(1, 1, 1)}


def test_radius_is_the_odd_side_nearest_sigma():
    for s in O.level_schedule():
        h = O.cross_level_radius(s["sigma"])
        side = 2 * h + 1
        assert side >= 3
        if s["sigma"] >= 2.0:
            assert abs(side - s["sigma"]) <= 1.0
    assert O.cross_level_radius(1.6) == 1 and O.cross_level_radius(21.0) == 10
    assert O.cross_level_radius(4.0) == 2 and O.cross_level_radius(3.9) == 1
