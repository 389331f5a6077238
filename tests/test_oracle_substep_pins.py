"""Pins of the oracle's sub-steps per level (level_step): closed forms on the
DCT-II basis when g is identically 1 (AOS and FED), convergence to a fine
explicit solution of the nonlinear equation as the number of sub-steps
grows (a conductivity held fixed over the level instead would stall), and
the reduction to the plain method at one sub-step."""
import numpy as np
import pytest
from scipy.fft import dctn, idctn

import oracle as O

K_FLAT = 1e30  # g2 = 1/(1 + m/k^2) rounds to exactly 1


def lam(n):
    return 4.0 * np.sin(np.pi * np.arange(n) / (2.0 * n)) ** 2


def spectral(L, factor):
    return idctn(dctn(L, type=2, norm="ortho") * factor, type=2, norm="ortho")


@pytest.mark.parametrize("m", [1, 2, 3, 7])
def test_aos_substeps_closed_form_for_unit_conductivity(m):
    rng = np.random.default_rng(m)
    H, W = 13, 17
    L = rng.random((H, W))
    tau = 23.5
    s = tau / m
    lx, ly = lam(W)[None, :], lam(H)[:, None]
    step = 0.5 * (1.0 / (1.0 + 2.0 * s * lx) + 1.0 / (1.0 + 2.0 * s * ly))
    ref = spectral(L, step ** m)
    got = O.level_step(L, K_FLAT, tau, "aos", m)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("m", [1, 2, 5])
def test_fed_substeps_closed_form_for_unit_conductivity(m):
    rng = np.random.default_rng(10 + m)
    H, W = 11, 14
    L = rng.random((H, W))
    tau = 31.0
    mu = -(lam(W)[None, :] + lam(H)[:, None])
    cyc = np.ones_like(mu)
    for t in O.fed_step_sizes(tau / m):
        cyc = cyc * (1.0 + t * mu)
    ref = spectral(L, cyc ** m)
    got = O.level_step(L, K_FLAT, tau, "fed", m)
    assert np.max(np.abs(got - ref)) < 1e-11


def test_substeps_converge_to_the_nonlinear_flow():
    """Against explicit Euler steps of dt = 0.01 with g recomputed at every
    step: the AOS error falls about like 1/m; holding the level's starting
    conductivity over all m sub-steps leaves an error that does not."""
    from synthetic import kaze_image
    L = O.gaussian_smooth(kaze_image(24, 20, 7).astype(np.float64), 1.6)
    k = O.contrast_factor(L)
    tau, dt = 4.0, 0.01
    ref = L.copy()
    for _ in range(int(round(tau / dt))):
        ref = ref + dt * O.diffusion_operator(ref, O.conductivity_g2(ref, k))
    ms = (1, 2, 4, 8, 16, 32)
    errs = [float(np.max(np.abs(O.level_step(L, k, tau, "aos", m) - ref))) for m in ms]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    # first order from m = 4 on: each doubling about halves the error
    assert all(1.6 < a / b < 2.2 for a, b in zip(errs[2:], errs[3:]))
    assert errs[-1] < errs[0] / 10
    g0 = O.conductivity_g2(L, k)
    frozen = L.copy()
    for _ in range(32):
        frozen = O.aos_step(frozen, g0, tau / 32)
    assert np.max(np.abs(frozen - ref)) > 4 * errs[-1]


def test_one_substep_is_the_plain_method():
    from synthetic import kaze_image
    img = kaze_image(40, 30, 3).astype(np.float64)
    a, ka = O.build_scale_space(img)
    b, kb = O.build_scale_space(img, substeps=1)
    assert ka == kb and np.array_equal(a, b)
    c, _ = O.build_scale_space(img, substeps=2)
    assert np.array_equal(a[0], c[0]) and not np.array_equal(a[1:], c[1:])
    with pytest.raises(ValueError):
        O.level_step(img, 0.1, 1.0, "aos", 0)
    with pytest.raises(ValueError):
        O.level_step(img, 0.1, 1.0, "explicit", 1)
