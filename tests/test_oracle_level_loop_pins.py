"""Pins of the oracle's level loop (build_scale_space) against closed forms.

The loop itself (which image level 0 is, the step length between levels, the
image the contrast factor is taken from) is checked here against facts fixed
by the paper and by linear algebra, computed in this file without the
oracle's schedule or filters:

* Sec. III-A: level 0 is the input smoothed by a Gaussian of sigma0 (here
  scipy.ndimage's Gaussian with the same radius, 5 = ceil(3 * 1.6), and the
  half-sample reflection, scipy's "reflect").
* Eqs. 6-7: sigma_i = sigma0 * 2**(i/S) for level i = o*S + s (the reading
  sigma0 * 2**(o + s/S)), t_i = sigma_i^2 / 2, and the step into level i has
  length tau_i = t_i - t_{i-1} = (sigma_i^2 - sigma_{i-1}^2) / 2.
* Eq. 4 by AOS with unit conductivity (k -> infinity makes g = 1 exactly in
  float64): each 1-D Neumann operator (I - 2 tau A) has the orthonormal
  DCT-II vectors as eigenvectors, with eigenvalues 1 + 2 tau lambda_k,
  lambda_k = 4 sin^2(pi k / (2 n)).  The AOS step therefore multiplies the
  2-D DCT-II coefficient (ky, kx) of the previous level by
  (1/(1 + 2 tau lambda_x[kx]) + 1/(1 + 2 tau lambda_y[ky])) / 2.
* Sec. II-A, III-A: the contrast factor is taken from the base image, level
  0, not from the raw input.

A loop with tau_i = t_i, an index shifted by one level, an unsmoothed level 0
or k taken from the raw image fails at least one of these tests.
"""
import numpy as np
import scipy.fft
import scipy.ndimage as ndi

import oracle as O
from synthetic import kaze_image

SIGMA0 = 1.6
OCTAVES = 4
SUBLEVELS = 4


def _base_image(img):
    # radius int(truncate * sigma + 0.5) = 5 = ceil(3 * 1.6)
    return ndi.gaussian_filter(np.asarray(img, dtype=np.float64), SIGMA0,
                               mode="reflect", truncate=5.0 / SIGMA0)


def _linear_aos_levels(L0, n_levels):
    """Levels 0..n_levels-1 of the scale space with g = 1, from the DCT."""
    H, W = L0.shape
    lam_x = 4.0 * np.sin(np.pi * np.arange(W) / (2.0 * W)) ** 2
    lam_y = 4.0 * np.sin(np.pi * np.arange(H) / (2.0 * H)) ** 2
    sig = [SIGMA0 * 2.0 ** (i / SUBLEVELS) for i in range(n_levels)]
    out = [L0]
    c = scipy.fft.dctn(L0, type=2, norm="ortho")
    for i in range(1, n_levels):
        tau = 0.5 * (sig[i] ** 2 - sig[i - 1] ** 2)
        mult = 0.5 * (1.0 / (1.0 + 2.0 * tau * lam_x[None, :])
                      + 1.0 / (1.0 + 2.0 * tau * lam_y[:, None]))
        c = c * mult
        out.append(scipy.fft.idctn(c, type=2, norm="ortho"))
    return np.stack(out)


def test_level_loop_with_unit_conductivity_is_the_dct_closed_form():
    img = kaze_image(41, 29, seed=11, n_blobs=6, n_shapes=4).astype(np.float64)
    levels, k = O.build_scale_space(img, sigma0=SIGMA0, octaves=OCTAVES,
                                    sublevels=SUBLEVELS, k=1e30)
    assert k == 1e30
    ref = _linear_aos_levels(_base_image(img), OCTAVES * SUBLEVELS)
    assert levels.shape == ref.shape
    for i in range(levels.shape[0]):
        err = np.max(np.abs(levels[i] - ref[i]))
        assert err <= 1e-12, (i, err)


def test_level_times_are_sigma_squared_over_two():
    """The level reached after i steps has diffused for t_i - t_0: with g = 1
    the DCT coefficient of the lowest nonzero frequency along x (on an image
    constant along y) is multiplied by the product of 1/(1 + 2 tau_j lam)
    over j <= i; recover each tau_j from consecutive levels."""
    W, H = 16, 5
    x = np.arange(W)
    img = np.tile(np.cos(np.pi * (x + 0.5) / W), (H, 1))   # DCT-II vector k = 1
    levels, _ = O.build_scale_space(img, sigma0=SIGMA0, octaves=OCTAVES,
                                    sublevels=SUBLEVELS, k=1e30)
    lam = 4.0 * np.sin(np.pi / (2.0 * W)) ** 2
    # along y the image is constant, so u_y = L and the AOS step multiplies
    # the mode by (1/(1 + 2 tau lam) + 1) / 2
    a = np.array([levels[i][2, 3] / levels[i - 1][2, 3] for i in range(1, 16)])
    tau = ((1.0 / (2.0 * a - 1.0)) - 1.0) / (2.0 * lam)
    t = [0.5 * (SIGMA0 * 2.0 ** (i / SUBLEVELS)) ** 2 for i in range(16)]
    expect = np.diff(t)
    assert np.max(np.abs(tau - expect) / expect) < 1e-9, (tau, expect)


def test_contrast_factor_is_taken_from_the_base_image():
    img = kaze_image(41, 29, seed=12, n_blobs=6, n_shapes=4).astype(np.float64)
    _, k = O.build_scale_space(img, sigma0=SIGMA0, octaves=1, sublevels=2)
    k_base = O.contrast_factor(_base_image(img), 1.0, 0.7, 300)
    k_raw = O.contrast_factor(img, 1.0, 0.7, 300)
    assert abs(k - k_base) <= 1e-12 * k_base
    # the raw image's k differs on this input, so the check above separates them
    assert abs(k_raw - k_base) > 1e-3 * k_base
