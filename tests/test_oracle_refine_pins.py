"""Pins of the oracle's keypoint refinement (Sec. II-B, Eqs. 9-12) against
facts that do not come from it: a generic least-squares solver on the 3x3
design, exact recovery of sampled quadratics and of their maximum, the
eigenvalues of the Hessian, and detector responses of synthetic blobs and
ridges with known centres."""
import numpy as np
import pytest

import oracle as O

U1 = np.array([-1.0, 0.0, 1.0])


def sample(a, b, c, d, e, f):
    U, V = np.meshgrid(U1, U1)
    return a + b * U + c * V + d * U * U + e * V * V + f * U * V


def test_fit_equals_generic_least_squares():
    rng = np.random.default_rng(31)
    U, V = np.meshgrid(U1, U1)
    A = np.stack([np.ones(9), U.ravel(), V.ravel(), (U * U).ravel(), (V * V).ravel(),
                  (U * V).ravel()], axis=1)
    for _ in range(50):
        p = rng.normal(size=(3, 3))
        ref = np.linalg.lstsq(A, p.ravel(), rcond=None)[0]
        assert np.allclose(O.quadratic_fit_3x3(p), ref, rtol=0, atol=1e-13)


def test_sampled_quadratic_and_its_maximum_are_recovered():
    rng = np.random.default_rng(32)
    for _ in range(50):
        # a negative definite quadratic whose maximum lies inside the window
        Hm = -np.diag(rng.uniform(0.5, 2.0, 2))
        R = np.linalg.qr(rng.normal(size=(2, 2)))[0]
        Hm = R @ Hm @ R.T
        x0 = rng.uniform(-0.9, 0.9, 2)
        peak = rng.uniform(0.01, 0.1)
        g = -Hm @ x0
        a = peak + 0.5 * x0 @ Hm @ x0
        coef = (a, g[0], g[1], Hm[0, 0] / 2, Hm[1, 1] / 2, Hm[0, 1])
        p = sample(*coef)
        assert np.allclose(O.quadratic_fit_3x3(p), coef, atol=1e-13)
        det = np.zeros((3, 5, 5))
        det[1, 1:4, 1:4] = p
        r = O.refine_keypoints(det, np.array([[1, 2, 2, p[1, 1]]]), edge_ratio=1e9)[0]
        assert np.allclose([r[2] - 2, r[1] - 2], x0, atol=1e-12)
        assert abs(r[3] - peak) < 1e-13
        assert r[5] == 1.0


def test_edge_ratio_is_the_eigenvalue_ratio_form():
    rng = np.random.default_rng(33)
    for _ in range(50):
        coef = rng.normal(size=6)
        a, b, c, d, e, f = coef
        H = np.array([[2 * d, f], [f, 2 * e]])
        det = np.zeros((3, 5, 5))
        det[1, 1:4, 1:4] = sample(*coef)
        r = O.refine_keypoints(det, np.array([[1, 2, 2, 0.0]]))[0]
        al, be = np.linalg.eigvalsh(H)
        if al * be > 0:
            assert np.isclose(r[4], (al + be) ** 2 / (al * be), rtol=1e-12)
        else:
            assert r[4] == np.inf and r[5] == 0.0


@pytest.mark.parametrize("ratio,kept", [(9.5, 1.0), (10.5, 0.0)])
def test_edge_threshold_at_r(ratio, kept):
    """Eigenvalue ratio just below / above r = 10: kept / rejected."""
    det = np.zeros((3, 5, 5))
    det[1, 1:4, 1:4] = sample(0.05, 0.0, 0.0, -ratio / 2 * 0.01, -0.5 * 0.01, 0.0)
    assert O.refine_keypoints(det, np.array([[1, 2, 2, 0.05]]))[0][5] == kept


def test_saddles_and_minima_are_rejected():
    det = np.zeros((3, 5, 5))
    det[1, 1:4, 1:4] = sample(0.05, 0.0, 0.0, -0.01, 0.01, 0.0)   # saddle
    assert O.refine_keypoints(det, np.array([[1, 2, 2, 0.05]]))[0][5] == 0.0
    det[1, 1:4, 1:4] = sample(0.05, 0.0, 0.0, 0.01, 0.01, 0.0)    # minimum
    assert O.refine_keypoints(det, np.array([[1, 2, 2, 0.05]]))[0][5] == 0.0


def blob_level(W, H, cx, cy, sx, sy):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return 0.5 + 0.4 * np.exp(-((x - cx) ** 2 / (2 * sx ** 2) + (y - cy) ** 2 / (2 * sy ** 2)))


def test_blob_centre_to_a_tenth_of_a_pixel():
    """A round blob centred between pixels: its detector response peaks at
    the nearest pixel and the refinement moves it towards the true centre."""
    W = H = 48
    for cx, cy in ((24.3, 23.8), (23.55, 24.4), (24.0, 24.0)):
        lev = np.stack([blob_level(W, H, cx, cy, 3.0, 3.0)] * 16)
        det = O.detector_response(lev)[:3]
        kp = O.find_extrema(np.stack([det[1] * 0.5, det[1], det[1] * 0.5]), 1e-6)
        assert len(kp) == 1
        r = O.refine_keypoints(np.stack([det[1] * 0.5, det[1], det[1] * 0.5]), kp)[0]
        assert r[5] == 1.0
        assert abs(r[2] - cx) < 0.1 and abs(r[1] - cy) < 0.1


@pytest.mark.parametrize("sx,sy,kept", [(8.0, 1.5, 0.0), (12.0, 1.5, 0.0), (3.0, 3.0, 1.0),
                                        (3.6, 3.0, 1.0)])
def test_ridges_are_rejected_and_blobs_kept(sx, sy, kept):
    """The extremum at the centre of an elongated blob fails the edge test of
    Eq. 12; round and mildly elongated blobs pass it."""
    W = H = 64
    lev = blob_level(W, H, 32.0, 32.0, sx, sy)
    det = O.detector_response(np.stack([lev] * 16))[:3]
    d = np.stack([det[1] * 0.5, det[1], det[1] * 0.5])
    kp = O.find_extrema(d, 1e-6)
    centre = kp[(np.abs(kp[:, 1] - 32) <= 1) & (np.abs(kp[:, 2] - 32) <= 1)]
    assert len(centre) == 1
    r = O.refine_keypoints(d, centre)[0]
    assert r[5] == kept
    assert (r[4] > (O.EDGE_RATIO + 1) ** 2 / O.EDGE_RATIO) == (kept == 0.0)
