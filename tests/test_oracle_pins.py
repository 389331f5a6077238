"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one part of the oracle against a closed form, an invariant
of the method, a brute-force loop written independently here, or an
independent library routine (scipy.ndimage, scipy.fft, numpy.linalg).
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.ndimage as ndi

import oracle as O
from synthetic import kaze_image


def _reflect(i, n):
    """Half-sample symmetric index: -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2."""
    p = 2 * n
    i = i % p
    return i if i < n else p - 1 - i


def _rand(H, W, seed):
    return np.random.default_rng(seed).random((H, W))


# ---------------------------------------------------------------- schedule
def test_schedule_closed_form():
    sch = O.level_schedule(1.6, 4, 4)
    assert len(sch) == 16
    assert sch[0]["sigma"] == pytest.approx(1.6, rel=0, abs=1e-15)
    for i in range(12):
        assert sch[i + 4]["sigma"] == pytest.approx(2 * sch[i]["sigma"], rel=1e-15)
    for lev in sch:
        assert lev["t"] == pytest.approx(lev["sigma"] ** 2 / 2, rel=1e-15)
        assert lev["o"] == lev["i"] // 4 and lev["s"] == lev["i"] % 4
        # normalised scale is periodic in the octave (Eq. 8)
        sn = lev["sigma"] / 2 ** lev["o"]
        assert sn == pytest.approx(1.6 * 2 ** (lev["s"] / 4), rel=1e-14)
    # strictly increasing evolution times
    ts = [lev["t"] for lev in sch]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert [O.derivative_step(1.6 * 2 ** (s / 4)) for s in range(4)] == [2, 2, 2, 3]


# ---------------------------------------------------------------- Gaussian
@pytest.mark.parametrize("sigma", [0.7, 1.0, 1.6, 2.3])
def test_gaussian_taps(sigma):
    w = O.gaussian_taps(sigma)
    r = int(math.ceil(3 * sigma))
    assert len(w) == 2 * r + 1
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w, w[::-1], atol=0)
    assert np.argmax(w) == r


@pytest.mark.parametrize("sigma", [1.0, 1.6])
def test_gaussian_matches_scipy_ndimage(sigma):
    img = _rand(37, 53, 3)
    r = int(math.ceil(3 * sigma))
    # scipy radius = int(truncate*sigma + 0.5); pick truncate so it equals r
    ref = ndi.gaussian_filter(img, sigma, mode="reflect", truncate=r / sigma)
    assert np.max(np.abs(O.gaussian_smooth(img, sigma) - ref)) < 1e-14


def test_gaussian_brute_force_2d_and_invariants():
    img = _rand(9, 11, 4)
    sigma = 1.6
    w = O.gaussian_taps(sigma)
    r = len(w) // 2
    H, W = img.shape
    ref = np.zeros_like(img)
    for y in range(H):
        for x in range(W):
            acc = 0.0
            for j in range(-r, r + 1):
                for i in range(-r, r + 1):
                    acc += w[j + r] * w[i + r] * img[_reflect(y + j, H), _reflect(x + i, W)]
            ref[y, x] = acc
    out = O.gaussian_smooth(img, sigma)
    assert np.max(np.abs(out - ref)) < 1e-14
    # half-sample reflection preserves the total
    assert out.sum() == pytest.approx(img.sum(), rel=1e-13)
    assert np.allclose(O.gaussian_smooth(np.full((8, 10), 0.37), sigma), 0.37, atol=1e-15)


# ---------------------------------------------------------------- Scharr
def test_scharr_against_kernel_and_ramp():
    img = _rand(12, 15, 5)
    kx = np.array([[-3, 0, 3], [-10, 0, 10], [-3, 0, 3]], dtype=np.float64) / 32.0
    assert np.max(np.abs(O.scharr_dx(img) - ndi.correlate(img, kx, mode="reflect"))) < 1e-15
    assert np.max(np.abs(O.scharr_dy(img) - ndi.correlate(img, kx.T, mode="reflect"))) < 1e-15
    yy, xx = np.mgrid[0:20, 0:24].astype(np.float64)
    a, b = 0.37, -1.25
    f = a * xx + b * yy
    for s in (1, 2, 3):
        inner = (slice(s, 20 - s), slice(s, 24 - s))
        assert np.allclose(O.scharr_dx(f, s)[inner], a, atol=1e-13)
        assert np.allclose(O.scharr_dy(f, s)[inner], b, atol=1e-13)


def test_scharr_step_brute_force():
    img = _rand(10, 13, 6)
    H, W = img.shape
    s = 2
    ref = np.zeros_like(img)
    for y in range(H):
        for x in range(W):
            acc = 0.0
            for dy, wy in ((-s, 3.0), (0, 10.0), (s, 3.0)):
                yy = _reflect(y + dy, H)
                acc += wy * (img[yy, _reflect(x + s, W)] - img[yy, _reflect(x - s, W)])
            ref[y, x] = acc / (32.0 * s)
    assert np.max(np.abs(O.scharr_dx(img, s) - ref)) < 1e-15
    assert np.max(np.abs(O.scharr_dy(img.T, s).T - ref)) < 1e-15


# ---------------------------------------------------------------- k and g
def test_contrast_factor_brackets_the_exact_quantile():
    img = kaze_image(96, 80, 11).astype(np.float64)
    L0 = O.gaussian_smooth(img, 1.6)
    k = O.contrast_factor(L0, 1.0, 0.7, 300)
    m = np.sort(O.gradient_magnitude(L0, 1.0).ravel())
    pos = m[m > 0]
    hmax = pos[-1]
    q = pos[int(math.ceil(0.7 * pos.size)) - 1]     # smallest value with >= 70% at or below it
    assert k - hmax / 300 - 1e-15 <= q <= k + 1e-15
    # flat image: no positive gradient, k falls back to 1
    assert O.contrast_factor(np.full((16, 16), 0.5)) == 1.0


def test_conductivity_special_values():
    yy, xx = np.mgrid[0:40, 0:40].astype(np.float64)
    k = 0.02
    ramp = k * xx                     # |grad| = k in the interior after smoothing
    g = O.conductivity_g2(ramp, k)
    assert np.allclose(g[6:-6, 6:-6], 0.5, atol=1e-12)
    g1 = O.conductivity_g1(ramp, k)
    assert np.allclose(g1[6:-6, 6:-6], math.exp(-1.0), atol=1e-12)
    assert np.all(O.conductivity_g2(np.full((12, 12), 0.3), k) == 1.0)
    gr = O.conductivity_g2(kaze_image(64, 48, 2).astype(np.float64), 0.01)
    assert gr.min() > 0.0 and gr.max() <= 1.0


# ---------------------------------------------------------------- AOS
def _flux_operator(u, g):
    """Brute-force 1-D nonlinear diffusion: sum over neighbours k of
    (g_j + g_k)/2 * (u_k - u_j), no flux across the ends."""
    n = len(u)
    out = np.zeros(n)
    for j in range(n):
        for k in (j - 1, j + 1):
            if 0 <= k < n:
                out[j] += 0.5 * (g[j] + g[k]) * (u[k] - u[j])
    return out


def test_aos_line_solve_matches_dense_system():
    rng = np.random.default_rng(7)
    for n in (2, 3, 7, 13):
        g = rng.uniform(0.01, 1.0, n)
        L = rng.random(n)
        tau = 3.7
        # dense I - 2 tau A, with A the Jacobian of the flux operator
        A = np.stack([_flux_operator(np.eye(n)[j], g) for j in range(n)], axis=1)
        B = np.eye(n) - 2 * tau * A
        ref = np.linalg.solve(B, L)
        img = L[None, :]
        got = O.aos_solve_rows(img, g[None, :], tau)[0]
        assert np.max(np.abs(got - ref)) < 1e-12
        got_c = O.aos_solve_cols(img.T.copy(), g[:, None], tau)[:, 0]
        assert np.max(np.abs(got_c - ref)) < 1e-12


def test_aos_step_small_tau_limit_is_divergence_form():
    L = _rand(9, 12, 8)
    g = np.random.default_rng(9).uniform(0.05, 1.0, L.shape)
    H, W = L.shape
    div = np.zeros_like(L)
    for y in range(H):
        div[y] += _flux_operator(L[y], g[y])
    for x in range(W):
        div[:, x] += _flux_operator(L[:, x], g[:, x])
    errs = []
    for tau in (1e-3, 1e-4):
        d = (O.aos_step(L, g, tau) - L) / tau
        errs.append(np.max(np.abs(d - div)))
    assert errs[1] < 1e-3
    assert errs[1] < errs[0] / 5          # first-order convergence in tau


def test_aos_conservation_and_max_min():
    L = kaze_image(48, 40, 3).astype(np.float64)
    g = O.conductivity_g2(L, 0.02)
    for tau in (0.53, 11.99, 67.86):
        u = O.aos_step(L, g, tau)
        assert u.sum() == pytest.approx(L.sum(), rel=1e-13)
        assert u.min() >= L.min() - 1e-14 and u.max() <= L.max() + 1e-14
        ux = O.aos_solve_rows(L, g, tau)
        assert np.allclose(ux.sum(axis=1), L.sum(axis=1), rtol=1e-13, atol=0)


def test_constant_image_stays_constant():
    img = np.full((24, 31), 0.4321)
    lev, k = O.build_scale_space(img)
    assert k == 1.0
    assert np.max(np.abs(lev - 0.4321)) < 1e-14
    det = O.detector_response(lev)
    assert np.max(np.abs(det)) < 1e-20
    assert len(O.find_extrema(det)) == 0


def test_unit_conductivity_is_linear_diffusion_dct():
    """g = 1: each 1-D Neumann operator is diagonalised by the orthonormal
    DCT-II, with eigenvalues 1 + 8 tau sin^2(pi k / 2n)."""
    L = _rand(17, 23, 10)
    tau = 5.9985
    g = np.ones_like(L)
    H, W = L.shape
    lam_x = 1 + 8 * tau * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2
    lam_y = 1 + 8 * tau * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2
    ux = scipy.fft.idct(scipy.fft.dct(L, norm="ortho", axis=1) / lam_x[None, :],
                        norm="ortho", axis=1)
    uy = scipy.fft.idct(scipy.fft.dct(L, norm="ortho", axis=0) / lam_y[:, None],
                        norm="ortho", axis=0)
    assert np.max(np.abs(O.aos_solve_rows(L, g, tau) - ux)) < 1e-12
    assert np.max(np.abs(O.aos_solve_cols(L, g, tau) - uy)) < 1e-12
    assert np.max(np.abs(O.aos_step(L, g, tau) - 0.5 * (ux + uy))) < 1e-12


# ---------------------------------------------------------------- Hessian
def test_hessian_exact_on_quadratics():
    yy, xx = np.mgrid[0:40, 0:44].astype(np.float64)
    a, b, c = 0.013, -0.007, 0.011
    f = a * xx ** 2 + b * yy ** 2 + c * xx * yy + 0.2 * xx - 0.1 * yy
    levels = np.stack([f] * 16)
    det = O.detector_response(levels)
    for lev in O.level_schedule():
        sn = lev["sigma"] / 2 ** lev["o"]
        s = O.derivative_step(sn)
        inner = (slice(2 * s, 40 - 2 * s), slice(2 * s, 44 - 2 * s))
        expect = sn * sn * (4 * a * b - c * c)
        assert np.allclose(det[lev["i"]][inner], expect, rtol=1e-10, atol=1e-15)


def test_hessian_brute_force_border_rule():
    """Each derivative image is reflected at the border before the next one."""
    L = _rand(11, 14, 12)
    s = 2

    def dx(f):
        H, W = f.shape
        out = np.zeros_like(f)
        for y in range(H):
            for x in range(W):
                out[y, x] = sum(wy * (f[_reflect(y + dy, H), _reflect(x + s, W)]
                                      - f[_reflect(y + dy, H), _reflect(x - s, W)])
                                for dy, wy in ((-s, 3), (0, 10), (s, 3))) / (32 * s)
        return out

    def dy(f):
        return dx(f.T).T

    Lx, Ly = dx(L), dy(L)
    ref = dx(Lx) * dy(Ly) - dy(Lx) ** 2
    levels = np.stack([L] * 16)
    det = O.detector_response(levels)
    sn = 1.6 * 2 ** (2 / 4)                    # level 2: step 2
    assert np.max(np.abs(det[2] - sn * sn * ref)) < 1e-15


# ---------------------------------------------------------------- extrema
def _brute_extrema(det, thr):
    N, H, W = det.shape
    out = []
    for i in range(1, N - 1):
        for y in range(1, H - 1):
            for x in range(1, W - 1):
                v = det[i, y, x]
                if not v > thr:
                    continue
                ok = True
                for dl in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            if (dl, dy, dx) != (0, 0, 0) and not v > det[i + dl, y + dy, x + dx]:
                                ok = False
                if ok:
                    out.append((i, y, x))
    return out


def test_extrema_brute_force_and_planted():
    rng = np.random.default_rng(13)
    det = rng.random((6, 9, 10)) * 0.01
    got = [tuple(int(v) for v in r[:3]) for r in O.find_extrema(det, 0.001)]
    assert got == _brute_extrema(det, 0.001)
    assert len(got) > 0
    flat = np.zeros((5, 12, 12))
    flat[2, 6, 5] = 0.5                        # isolated peak
    flat[3, 3, 3] = flat[3, 3, 4] = 0.4        # plateau: a tie is not a maximum
    assert [tuple(int(v) for v in r[:3]) for r in O.find_extrema(flat, 0.001)] == [(2, 6, 5)]
    below = np.zeros((5, 12, 12))
    below[2, 6, 5] = 0.001                     # at the threshold: strict, not found
    assert len(O.find_extrema(below, 0.001)) == 0
    edge = np.zeros((5, 12, 12))
    edge[2, 0, 5] = edge[2, 6, 11] = edge[0, 6, 6] = edge[4, 5, 5] = 0.5
    assert len(O.find_extrema(edge, 0.001)) == 0


# ---------------------------------------------------------------- symmetry
def test_transpose_and_mirror_symmetry():
    img = kaze_image(40, 32, 21).astype(np.float64)
    lev, k = O.build_scale_space(img)
    levT, kT = O.build_scale_space(img.T.copy())
    assert kT == pytest.approx(k, rel=1e-12)
    assert np.max(np.abs(levT - lev.transpose(0, 2, 1))) < 1e-12
    levM, kM = O.build_scale_space(img[:, ::-1].copy())
    assert np.max(np.abs(levM - lev[:, :, ::-1])) < 1e-12
    det = O.detector_response(lev)
    detT = O.detector_response(levT)
    # L_xy = D_y(D_x L) with each derivative image reflected: D_x and D_y
    # commute everywhere except within one step (<= 3 px) of the border
    m = 3
    assert np.max(np.abs(detT - det.transpose(0, 2, 1))[:, m:-m, m:-m]) < 1e-14
    detM = O.detector_response(levM)
    assert np.max(np.abs(detM - det[:, :, ::-1])) < 1e-14


def test_single_blob_keypoint_at_centre():
    H = W = 65
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = 0.3 + 0.5 * np.exp(-((xx - 32) ** 2 + (yy - 32) ** 2) / (2 * 4.0 ** 2))
    lev, k = O.build_scale_space(img)
    det = O.detector_response(lev)
    kps = O.find_extrema(det, 1e-6)
    assert len(kps) >= 1
    centres = {(int(r[1]), int(r[2])) for r in kps}
    assert centres == {(32, 32)}
