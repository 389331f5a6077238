"""Pins of the oracle's FED cycle (Eq. 5) against facts that do not come from
it: the closed-form cycle length of the FED step sizes, a brute-force flux
loop, the DCT diagonalisation of the g = 1 operator, the stability of the
cycle polynomial, conservation, and second-order agreement with the AOS
step for small steps."""
import numpy as np
import pytest
from scipy.fft import dctn, idctn

import oracle as O
from synthetic import kaze_image


def test_cycle_length_closed_form_and_minimal_n():
    """Unscaled Eq. 5 steps of a cycle of n sum to tau_max (n^2 + n) / 3
    (Grewenig et al. 2010); the oracle picks the smallest such n >= T."""
    tm = O.FED_TAU_MAX
    for n in range(1, 41):
        j = np.arange(n)
        raw = tm / (2 * np.cos(np.pi * (2 * j + 1) / (4 * n + 2)) ** 2)
        assert np.isclose(raw.sum(), tm * (n * n + n) / 3.0, rtol=1e-12)
    for T in [0.01, 0.1, 0.5302, 0.75, 1.06, 5.99, 23.99, 67.86]:
        t = O.fed_step_sizes(T)
        n = len(t)
        assert np.isclose(t.sum(), T, rtol=1e-14)
        assert tm * (n * n + n) / 3.0 >= T
        assert n == 1 or tm * ((n - 1) ** 2 + (n - 1)) / 3.0 < T


def brute_operator(L, g):
    H, W = L.shape
    out = np.zeros_like(L)
    for y in range(H):
        for x in range(W):
            s = 0.0
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W:
                    s += 0.5 * (g[y, x] + g[yy, xx]) * (L[yy, xx] - L[y, x])
            out[y, x] = s
    return out


def test_operator_and_single_step_by_brute_force():
    rng = np.random.default_rng(21)
    L = rng.uniform(0, 1, size=(7, 9))
    g = rng.uniform(0.05, 1, size=(7, 9))
    assert np.allclose(O.diffusion_operator(L, g), brute_operator(L, g), rtol=0, atol=1e-14)
    T = 0.1   # below 2 tau_max / 3: a single explicit step of size T
    assert len(O.fed_step_sizes(T)) == 1
    assert np.allclose(O.fed_cycle(L, g, T), L + T * brute_operator(L, g), rtol=0, atol=1e-14)


@pytest.mark.parametrize("T", [0.53, 4.24, 67.86])
def test_g1_cycle_is_the_dct_polynomial(T):
    """With g = 1 the operator is diagonal in the orthonormal DCT-II basis with
    eigenvalues -4 sin^2(pi k / 2H) - 4 sin^2(pi l / 2W); a cycle multiplies
    each coefficient by prod_j (1 + tau_j mu)."""
    H, W = 12, 17
    L = kaze_image(W, H, 22).astype(np.float64)
    g = np.ones_like(L)
    k = np.arange(H)[:, None]
    l = np.arange(W)[None, :]
    mu = -4 * np.sin(np.pi * k / (2 * H)) ** 2 - 4 * np.sin(np.pi * l / (2 * W)) ** 2
    P = np.ones_like(mu)
    for t in O.fed_step_sizes(T):
        P *= 1 + t * mu
    ref = idctn(P * dctn(L, norm="ortho"), norm="ortho")
    assert np.allclose(O.fed_cycle(L, g, T), ref, rtol=0, atol=1e-11)


def test_cycle_polynomial_is_stable():
    """|prod_j (1 + tau_j mu)| <= 1 over the whole spectrum [-8, 0] of the
    g <= 1 operator, for every step size of the default schedule."""
    mu = np.linspace(-8.0, 0.0, 20001)
    for T in [0.5302, 0.7498, 1.0604, 1.4996, 2.1208, 2.9992, 4.2415, 5.9985, 8.4831,
              11.9969, 16.9662, 23.9938, 33.9324, 47.9876, 67.8648]:
        P = np.ones_like(mu)
        for t in O.fed_step_sizes(T):
            P *= 1 + t * mu
        assert np.max(np.abs(P)) <= 1 + 1e-9, T


def test_conservation_and_constants():
    img = kaze_image(30, 22, 23).astype(np.float64)
    g = O.conductivity_g2(img, 0.05)
    out = O.fed_cycle(img, g, 16.97)
    assert np.isclose(out.sum(), img.sum(), rtol=1e-12)
    c = np.full((9, 11), 0.37)
    assert np.allclose(O.fed_cycle(c, O.conductivity_g2(c, 0.05), 5.0), 0.37, atol=1e-15)


def test_fed_and_aos_agree_to_second_order_for_small_steps():
    """Both are consistent first-order schemes of the same semi-discrete PDE:
    their difference after one step T shrinks like T^2."""
    img = kaze_image(40, 30, 24).astype(np.float64)
    g = O.conductivity_g2(O.gaussian_smooth(img, 1.6), 0.03)
    L = O.gaussian_smooth(img, 1.6)
    d = []
    for T in (0.08, 0.04, 0.02):
        d.append(np.abs(O.fed_cycle(L, g, T) - O.aos_step(L, g, T)).max())
    assert 3.0 < d[0] / d[1] < 5.0 and 3.0 < d[1] / d[2] < 5.0


def test_scale_space_with_fed():
    img = kaze_image(48, 36, 25).astype(np.float64)
    lev_f, k_f = O.build_scale_space(img, scheme="fed")
    lev_a, k_a = O.build_scale_space(img)
    assert k_f == k_a and np.array_equal(lev_f[0], lev_a[0])
    # same PDE, different time integration: close but not equal
    diff = np.abs(lev_f - lev_a).max(axis=(1, 2))
    assert np.all(diff[1:] > 0) and np.all(diff < 0.1)
    assert np.allclose(lev_f.sum(axis=(1, 2)), lev_f[0].sum(), rtol=1e-12)


def test_step_order_is_a_permutation_and_order_free_in_exact_arithmetic():
    """The kappa order visits every step once; applied to the DCT
    coefficients (exact per frequency) any order gives the same cycle."""
    for T in (0.53, 5.99, 67.86):
        t = O.fed_step_sizes(T)
        order = O.fed_order(t)
        assert sorted(order.tolist()) == list(range(len(t)))
    mu = np.linspace(-8, 0, 101)
    t = O.fed_step_sizes(23.99)
    a = np.prod([1 + x * mu for x in t], axis=0)
    b = np.prod([1 + t[j] * mu for j in O.fed_order(t)], axis=0)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-15)
