"""FP64 CPU oracle of the KAZE nonlinear scale space and detector response.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke entry
point and the CPU-baseline leg of the benchmark may import this module.  It
shares no code, table or constant generator with the GPU library: it is a
plain, slow, readable restatement of the method of Ramkumar B et al., "GPGPU
Acceleration of the KAZE Image Feature Extraction Algorithm" (arXiv
1706.06750), Sec. II-A and II-B, in float64 NumPy.

Readings of passages the paper leaves open (each is also listed in the
design notes):

* Eq. 6 exponent: sigma_i = sigma0 * 2**(o + s/S) (the printed (o+s)/S would
  give duplicate scales and is not octave periodic, as Eq. 8 requires).
* N = O*S levels, i = 0..N-1; level 0 is the sigma0-smoothed base image
  (Sec. III-A), t_0 = sigma0^2/2; one semi-implicit step per level with
  tau_i = t_i - t_{i-1}.
* Eq. 4 is evaluated by additive operator splitting (AOS): for m = 2
  dimensions, L^{i} = 1/m sum_l (I - m tau A_l(L^{i-1}))^{-1} L^{i-1}, where A_l
  is the 1-D nonlinear diffusion matrix with entries (g_j + g_k)/2 between
  neighbours j,k (pixel spacing 1) and minus their sum on the diagonal.
  Neumann (zero-flux) boundaries drop the flux across the image border.
* All stencils extend the image by half-sample symmetric reflection
  (x[-1] = x[0], x[-2] = x[1], ...), the reflection consistent with the
  cell-centred Neumann boundary.
* Gaussian kernels: radius ceil(3 sigma), taps exp(-j^2/(2 sigma^2))
  normalised to sum 1.  The image used for the conductivity is smoothed with
  sigma_cond = 1.0 before the Scharr derivatives (Sec. III-A).
* Scharr derivatives at step s: central difference (f(x+s)-f(x-s))/(2s)
  across, [3, 10, 3]/16 smoothing at offsets (-s, 0, +s) along the other axis
  (s = 1 is the ordinary 3x3 Scharr kernel divided by 32).
* Contrast factor k (Sec. II-A, Sec. III-A): magnitudes of the Scharr
  gradient of the sigma_cond-smoothed base image over all pixels; zero
  magnitudes excluded; 300 bins over [0, hmax], bin = min(floor(m/hmax*300),
  299); b* = smallest bin whose cumulative count reaches 0.7 * npos;
  k = hmax * (b*+1)/300 (upper bin edge).  With no positive magnitude k = 1.
* Eq. 8: the scale factor is sigma_n,i = sigma_i / 2**o_i (the printed k_i
  reuses the contrast-factor symbol); the derivative step is round(sigma_n)
  (half away from zero); the det is weighted by the real sigma_n^2;
  L_xx = D_x(D_x L), L_yy = D_y(D_y L), L_xy = D_y(D_x L), each derivative
  image reflected at the border before the next derivative.
* Extrema (Sec. II-B, the 3x3 "approximate" variant): levels 1..N-2, pixels
  1..W-2 x 1..H-2, response strictly above the threshold and strictly above
  all 26 neighbours in the 3x3x3 block; maxima only.
* Extrema, the "exact" variant (Sec. II-B, Sec. III-B, Sec. IV): the same
  candidates (threshold, 3x3 maximum in their own level), which must also
  lie strictly above every response of levels i-1 and i+1 in a square
  window centred on them whose side is the odd number nearest sigma_i, at
  least 3: half-side h_i = max(1, round((sigma_i - 1) / 2)) with sigma_i the
  candidate level's scale of Eq. 6 (1 at the first levels, 10 at the last of
  the default 16).  Window pixels outside the image are left out.  With
  h_i = 1 this is the approximate variant, and every larger window only
  adds comparisons, so the exact set is a subset (as the paper observes).
* FED (Eq. 5, the scheme the paper's own GPU code runs): the step from
  t_{i-1} to t_i (length T = tau_i) is one cycle of n explicit steps
  L <- L + tau_j sum_l A_l(g) L with the same A_l as the AOS step and g
  computed once from L_{i-1}.  tau_max = 1/4, the stability limit of the 2-D
  explicit scheme with unit spacing and g <= 1; n is the smallest cycle
  length whose total time tau_max (n^2 + n)/3 reaches T, and the Eq. 5 step
  sizes are scaled by T over that total so the cycle ends exactly at t_i.
  With g fixed the n step operators commute, so their order changes only
  the rounding: in the order j = 0 .. n-1 the intermediate values of a
  29-step cycle grow by ~1e12.  The steps are applied in the order
  i -> kappa i mod n (the kappa-cycles of Grewenig et al. 2010), kappa
  coprime to n and chosen to minimise the error-growth bound
  max_k max|prod_{j<k}(1 + tau_j mu)| max|prod_{j>=k}(1 + tau_j mu)| over
  mu in [-8, 0] on a grid of 2001 points (ties: smallest kappa).
* Sub-steps per level (the stepping variant of the method's AOS form): with
  m sub-steps the level step of length tau_i is split into m equal steps of
  tau_i / m, each of which recomputes the conductivity from its own starting
  image and then takes one AOS step (or one FED cycle) of that length.  m = 1
  is the method as stated.
* Description stage (Sec. II-C, Sec. III-C).  The derivatives are the
  detector's first derivatives (Eq. 8's concatenated Scharr filter of step
  round(sigma_n)) scaled by sigma_n, Lx = sigma_n D_x L and Ly = sigma_n D_y L.
  The keypoint's scale unit is s = sigma_i of its level (Eq. 6, in pixels;
  no level is downsampled); the implementation section's "1.5 times the
  scale" conflicts with the method section and is not followed.  Samples
  at real positions are bilinear in Lx and Ly with pixel centres at integer
  coordinates and the half-sample reflection of the image, repeated with
  period 2n for positions more than one image away.
* Dominant orientation: samples at (x, y) + s (u, v) for integers u, v with
  u^2 + v^2 <= 36 (radius 6 s, step s: 113 samples), each response
  w (Lx, Ly) with w = exp(-(u^2 + v^2) / (2 * 2.5^2)) (a Gaussian of 2.5 s
  at the keypoint; the paper gives no width and 2.5 s is the descriptor's
  sigma_1), at the angle phi = atan2(w Ly, w Lx).  A sector of pi/3 slides
  round the circle; its sum changes only where an edge crosses a response,
  so every sum it takes is one of the sums over the half-open sectors
  (phi_k, phi_k + pi/3] and (phi_k - pi/3, phi_k], k = 1..113.  The
  orientation is the angle of the longest of these sums (ties: the first
  in the order k = 1.., "after" before "before").
* M-SURF descriptor: the 24 s x 24 s window centred on the keypoint and
  turned by the orientation theta has 4 x 4 subregions of 9 s x 9 s
  centred at -7.5, -2.5, 2.5, 7.5 (units of s) along and across theta, so
  neighbours overlap by 2 s on either side; each subregion is sampled on a
  9 x 9 grid of step s around its centre.  A sample at (u, v) lies at
  (x, y) + s (u cos theta - v sin theta, u sin theta + v cos theta); its
  derivatives along and across theta are d_u = Lx cos + Ly sin,
  d_v = -Lx sin + Ly cos, weighted by exp(-((u-c_u)^2 + (v-c_v)^2) /
  (2 * 2.5^2)) (sigma_1 = 2.5 s at the subregion centre) and summed into
  (sum d_u, sum d_v, sum |d_u|, sum |d_v|).  Each subregion's four sums are
  weighted by exp(-((a-1.5)^2 + (b-1.5)^2) / (2 * 1.5^2)) over the 4 x 4
  mask (sigma_2 = 1.5 in subregion units: in pixels it would weight the
  corner subregions by e^-25), ordered by subregion row b (across), column
  a (along), then the four sums, and the 64-vector is scaled to unit length
  (left zero if it is zero).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_banded

__all__ = [
    "DEFAULTS", "level_schedule", "gaussian_taps", "gaussian_smooth",
    "scharr_dx", "scharr_dy", "gradient_magnitude", "contrast_factor",
    "conductivity_g2", "conductivity_g1", "aos_line_bands", "aos_solve_rows",
    "aos_solve_cols", "aos_step", "build_scale_space", "derivative_step",
    "detector_response", "find_extrema", "cross_level_radius", "FED_TAU_MAX", "fed_step_sizes",
    "fed_order", "diffusion_operator", "explicit_step", "fed_cycle", "level_step",
    "EDGE_RATIO", "quadratic_fit_3x3", "refine_keypoints", "first_derivatives",
    "bilinear", "orientation_samples", "dominant_orientation", "msurf_descriptor",
    "describe_keypoints",
]

DEFAULTS = dict(sigma0=1.6, octaves=4, sublevels=4, sigma_cond=1.0,
                k_percentile=0.7, k_bins=300, det_threshold=0.001)


# --------------------------------------------------------------------------
# Scale schedule: Eqs. 6 and 7 (Sec. II-A)
# --------------------------------------------------------------------------
def level_schedule(sigma0: float = 1.6, octaves: int = 4, sublevels: int = 4):
    """Per level i: octave o, sublevel s, scale sigma_i and time t_i.

    Eq. 6 maps (o, s) to sigma_i = sigma0 * 2**(o + s/S) (read as KAZE's own
    definition); Eq. 7 converts it to the evolution time t_i = sigma_i^2 / 2.
    """
    out = []
    for o in range(octaves):
        for s in range(sublevels):
            sigma = sigma0 * 2.0 ** (o + s / sublevels)
            out.append({"i": len(out), "o": o, "s": s, "sigma": sigma,
                        "t": 0.5 * sigma * sigma})
    return out


# --------------------------------------------------------------------------
# Linear filters (Sec. III-A: Gaussian pre-smoothing, L_smooth, Scharr)
# --------------------------------------------------------------------------
def _extend(f: np.ndarray, r: int, axis: int) -> np.ndarray:
    """Half-sample symmetric extension by r samples on both sides of an axis."""
    pad = [(0, 0), (0, 0)]
    pad[axis] = (r, r)
    return np.pad(f, pad, mode="symmetric")


def _correlate_axis(f: np.ndarray, taps: np.ndarray, offsets, axis: int
                    ) -> np.ndarray:
    """out[p] = sum_j taps[j] * f[p + offsets[j] along axis], reflected border."""
    r = max(abs(int(o)) for o in offsets)
    n = f.shape[axis]
    fe = _extend(f, r, axis)
    out = np.zeros_like(f, dtype=np.float64)
    for w, o in zip(taps, offsets):
        sl = [slice(None), slice(None)]
        sl[axis] = slice(r + o, r + o + n)
        out += w * fe[tuple(sl)]
    return out


def gaussian_taps(sigma: float) -> np.ndarray:
    """Sampled Gaussian, radius ceil(3 sigma), normalised to unit sum."""
    r = int(math.ceil(3.0 * sigma))
    j = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(j * j) / (2.0 * sigma * sigma))
    return w / w.sum()


def gaussian_smooth(f: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian convolution G_sigma * f (Sec. III-A), x then y."""
    taps = gaussian_taps(sigma)
    r = len(taps) // 2
    offs = list(range(-r, r + 1))
    tmp = _correlate_axis(np.asarray(f, dtype=np.float64), taps, offs, axis=1)
    return _correlate_axis(tmp, taps, offs, axis=0)


def scharr_dx(f: np.ndarray, s: int = 1) -> np.ndarray:
    """Scharr x-derivative of step s (Sec. II-B; Sec. III-B concatenated form).

    Central difference (f(x+s) - f(x-s)) / (2s) along x, smoothed by
    [3, 10, 3]/16 at y offsets (-s, 0, +s).
    """
    d = _correlate_axis(np.asarray(f, dtype=np.float64),
                        [-1.0 / (2 * s), 1.0 / (2 * s)], [-s, s], axis=1)
    return _correlate_axis(d, [3 / 16, 10 / 16, 3 / 16], [-s, 0, s], axis=0)


def scharr_dy(f: np.ndarray, s: int = 1) -> np.ndarray:
    """Scharr y-derivative of step s: the transpose of :func:`scharr_dx`."""
    d = _correlate_axis(np.asarray(f, dtype=np.float64),
                        [-1.0 / (2 * s), 1.0 / (2 * s)], [-s, s], axis=0)
    return _correlate_axis(d, [3 / 16, 10 / 16, 3 / 16], [-s, 0, s], axis=1)


def gradient_magnitude(L: np.ndarray, sigma_cond: float = 1.0) -> np.ndarray:
    """|grad L_sigma|: Scharr gradient of G_sigma_cond * L (Eq. 2)."""
    Ls = gaussian_smooth(L, sigma_cond)
    Lx, Ly = scharr_dx(Ls), scharr_dy(Ls)
    return np.sqrt(Lx * Lx + Ly * Ly)


# --------------------------------------------------------------------------
# Contrast factor and conductivity: Eqs. 2-3, Sec. III-A
# --------------------------------------------------------------------------
def contrast_factor(L0: np.ndarray, sigma_cond: float = 1.0,
                    percentile: float = 0.7, nbins: int = 300) -> float:
    """Contrast factor k from the gradient histogram of the base image."""
    m = gradient_magnitude(L0, sigma_cond)
    pos = m[m > 0.0]
    if pos.size == 0:
        return 1.0
    hmax = float(m.max())
    bins = np.minimum(np.floor(pos / hmax * nbins).astype(np.int64), nbins - 1)
    hist = np.bincount(bins, minlength=nbins)
    cum = np.cumsum(hist)
    b = int(np.argmax(cum >= percentile * pos.size))
    return hmax * (b + 1) / nbins


def conductivity_g2(L: np.ndarray, k: float, sigma_cond: float = 1.0
                    ) -> np.ndarray:
    """Perona-Malik g2 = 1 / (1 + |grad L_sigma|^2 / k^2) (Eqs. 2-3)."""
    Ls = gaussian_smooth(L, sigma_cond)
    Lx, Ly = scharr_dx(Ls), scharr_dy(Ls)
    return 1.0 / (1.0 + (Lx * Lx + Ly * Ly) / (k * k))


def conductivity_g1(L: np.ndarray, k: float, sigma_cond: float = 1.0
                    ) -> np.ndarray:
    """Perona-Malik g1 = exp(-|grad L_sigma|^2 / k^2) (Eq. 3)."""
    Ls = gaussian_smooth(L, sigma_cond)
    Lx, Ly = scharr_dx(Ls), scharr_dy(Ls)
    return np.exp(-(Lx * Lx + Ly * Ly) / (k * k))


# --------------------------------------------------------------------------
# Semi-implicit step, Eq. 4, by additive operator splitting
# --------------------------------------------------------------------------
def aos_line_bands(g_line: np.ndarray, tau: float, m: int = 2) -> np.ndarray:
    """Banded form (scipy 'ab' layout) of I - m tau A(g) for one image line.

    A has (g_j + g_{j+1})/2 between neighbours j, j+1 and minus the row sum
    on the diagonal; the flux across either end of the line is dropped.
    """
    g = np.asarray(g_line, dtype=np.float64)
    n = g.size
    w = m * tau * 0.5 * (g[:-1] + g[1:])     # coupling weight of edge (j, j+1)
    ab = np.zeros((3, n), dtype=np.float64)
    ab[0, 1:] = -w                           # super-diagonal
    ab[2, :-1] = -w                          # sub-diagonal
    ab[1, :] = 1.0
    ab[1, :-1] += w
    ab[1, 1:] += w
    return ab


def aos_solve_rows(L: np.ndarray, g: np.ndarray, tau: float) -> np.ndarray:
    """u_x: (I - 2 tau A_x(g)) u_x = L along every row."""
    H, W = L.shape
    out = np.empty((H, W), dtype=np.float64)
    for y in range(H):
        if W == 1:
            out[y] = L[y]
            continue
        out[y] = solve_banded((1, 1), aos_line_bands(g[y], tau), L[y])
    return out


def aos_solve_cols(L: np.ndarray, g: np.ndarray, tau: float) -> np.ndarray:
    """u_y: (I - 2 tau A_y(g)) u_y = L along every column."""
    return aos_solve_rows(L.T, g.T, tau).T


def aos_step(L: np.ndarray, g: np.ndarray, tau: float) -> np.ndarray:
    """One AOS step of Eq. 4: L' = (u_x + u_y) / 2."""
    L = np.asarray(L, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    return 0.5 * (aos_solve_rows(L, g, tau) + aos_solve_cols(L, g, tau))


# --------------------------------------------------------------------------
# FED: Eq. 5
# --------------------------------------------------------------------------
FED_TAU_MAX = 0.25


def fed_step_sizes(T: float, tau_max: float = FED_TAU_MAX) -> np.ndarray:
    """Step sizes of one FED cycle of total time T (Eq. 5, scaled to T)."""
    if not (T > 0.0):
        raise ValueError("T must be > 0")
    n = 1
    while tau_max * (n * n + n) / 3.0 < T:
        n += 1
    j = np.arange(n, dtype=np.float64)
    tau = tau_max / (2.0 * np.cos(np.pi * (2.0 * j + 1.0) / (4.0 * n + 2.0)) ** 2)
    return tau * (T / tau.sum())


def fed_order(tau: np.ndarray) -> np.ndarray:
    """Application order of a cycle's steps: i -> kappa i mod n (see the
    module notes)."""
    n = len(tau)
    mu = np.linspace(-8.0, 0.0, 2001)
    best, best_k = None, 1
    for kappa in range(1, max(n, 2)):
        if math.gcd(kappa, n) != 1:
            continue
        order = [(kappa * i) % n for i in range(n)]
        pre = np.ones_like(mu)
        prefix = [1.0]
        for j in order:
            pre = pre * (1.0 + tau[j] * mu)
            prefix.append(np.abs(pre).max())
        suf = np.ones_like(mu)
        suffix = [1.0]
        for j in order[::-1]:
            suf = suf * (1.0 + tau[j] * mu)
            suffix.append(np.abs(suf).max())
        suffix = suffix[::-1]
        bound = max(a * b for a, b in zip(prefix, suffix))
        if best is None or bound < best * (1.0 - 1e-12):
            best, best_k = bound, kappa
    return np.array([(best_k * i) % n for i in range(n)], dtype=np.int64)


def diffusion_operator(L: np.ndarray, g: np.ndarray) -> np.ndarray:
    """sum_l A_l(g) L: the flux (g_j + g_k)/2 (L_k - L_j) from every
    neighbour k along rows and columns, none across the border."""
    L = np.asarray(L, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros_like(L)
    wx = 0.5 * (g[:, :-1] + g[:, 1:])
    fx = wx * (L[:, 1:] - L[:, :-1])
    out[:, :-1] += fx
    out[:, 1:] -= fx
    wy = 0.5 * (g[:-1, :] + g[1:, :])
    fy = wy * (L[1:, :] - L[:-1, :])
    out[:-1, :] += fy
    out[1:, :] -= fy
    return out


def explicit_step(L: np.ndarray, g: np.ndarray, tau: float) -> np.ndarray:
    return np.asarray(L, dtype=np.float64) + tau * diffusion_operator(L, g)


def fed_cycle(L: np.ndarray, g: np.ndarray, T: float) -> np.ndarray:
    """One FED cycle of total time T with the conductivity g held fixed."""
    out = np.asarray(L, dtype=np.float64)
    tau = fed_step_sizes(T)
    for j in fed_order(tau):
        out = explicit_step(out, g, tau[j])
    return out


# Keypoint refinement (Sec. II-B, Eqs. 9-12).
#
# Readings: the "two-dimensional quadratic function" fitted to the 3x3
# detector responses is the least-squares fit of
#   q(u, v) = a + b u + c v + d u^2 + e v^2 + f u v,   u, v in {-1, 0, 1},
# to the nine samples; its stationary point gives the sub-pixel offset and
# its value there the refined response.  The Hessian of Eqs. 9-12 ("from 8
# points around" the candidate) is that of the same quadratic,
# [[2d, f], [f, 2e]]; Eq. 10's trace is D_xx + D_yy (the printed D_xy is a
# typo); the ratio r of Eq. 12 is not given in the paper and is taken as 10,
# SIFT's value.  A candidate is kept when its Hessian is negative definite
# (a maximum), Tr(H)^2 / Det(H) < (r + 1)^2 / r and both offsets are at most
# one pixel.
EDGE_RATIO = 10.0


def quadratic_fit_3x3(p: np.ndarray):
    """Least-squares coefficients (a, b, c, d, e, f) of the quadratic above
    for a 3x3 patch p[v + 1][u + 1] (rows v, columns u).

    On the 3x3 grid the regressors 1, u, v, u^2 - 2/3, v^2 - 2/3 and u v are
    mutually orthogonal, so each coefficient is a projection."""
    p = np.asarray(p, dtype=np.float64)
    u = np.array([-1.0, 0.0, 1.0])
    U, V = np.meshgrid(u, u)          # U[v][u] = u, V[v][u] = v
    b = (p * U).sum() / (U * U).sum()
    c = (p * V).sum() / (V * V).sum()
    f = (p * U * V).sum() / (U * U * V * V).sum()
    Uc, Vc = U * U - 2.0 / 3.0, V * V - 2.0 / 3.0
    d = (p * Uc).sum() / (Uc * Uc).sum()
    e = (p * Vc).sum() / (Vc * Vc).sum()
    a = p.mean() - 2.0 / 3.0 * (d + e)
    return a, b, c, d, e, f


def refine_keypoints(det: np.ndarray, kps: np.ndarray, edge_ratio: float = EDGE_RATIO):
    """Sub-pixel position, refined response and edge test of every extremum.

    kps: (n, 4) rows (level, y, x, response) as from find_extrema.
    Returns (n, 6) float64 rows (level, y + dv, x + du, q(du, dv), ratio,
    kept) with ratio = Tr(H)^2 / Det(H) (inf when Det(H) <= 0) and kept 1.0
    or 0.0."""
    det = np.asarray(det, dtype=np.float64)
    out = []
    thr = (edge_ratio + 1.0) ** 2 / edge_ratio
    for lev, y, x, _ in np.asarray(kps, dtype=np.float64).reshape(-1, 4):
        lev, y, x = int(lev), int(y), int(x)
        a, b, c, d, e, f = quadratic_fit_3x3(det[lev, y - 1:y + 2, x - 1:x + 2])
        hxx, hyy, hxy = 2.0 * d, 2.0 * e, f
        dt = hxx * hyy - hxy * hxy
        tr = hxx + hyy
        ratio = tr * tr / dt if dt > 0.0 else np.inf
        if dt != 0.0:
            du = -(hyy * b - hxy * c) / dt
            dv = -(hxx * c - hxy * b) / dt
        else:
            du = dv = np.inf
        maximum = dt > 0.0 and tr < 0.0
        kept = maximum and ratio < thr and abs(du) <= 1.0 and abs(dv) <= 1.0
        if np.isfinite(du) and np.isfinite(dv):
            val = a + b * du + c * dv + d * du * du + e * dv * dv + f * du * dv
        else:
            val = np.nan
        out.append((lev, y + dv, x + du, val, ratio, 1.0 if kept else 0.0))
    return np.array(out, dtype=np.float64).reshape(-1, 6)


def level_step(L: np.ndarray, k: float, tau: float, scheme: str = "aos",
               substeps: int = 1, diffusivity: str = "g2", sigma_cond: float = 1.0):
    """The step from one level to the next, of total length tau: ``substeps``
    equal steps, each with the conductivity (Eqs. 2-3) of its own starting
    image, by AOS (Eq. 4) or by one FED cycle (Eq. 5)."""
    if scheme not in ("aos", "fed"):
        raise ValueError("scheme must be 'aos' or 'fed'")
    if substeps < 1:
        raise ValueError("substeps must be >= 1")
    cond = conductivity_g2 if diffusivity == "g2" else conductivity_g1
    out = np.asarray(L, dtype=np.float64)
    for _ in range(substeps):
        g = cond(out, k, sigma_cond)
        out = aos_step(out, g, tau / substeps) if scheme == "aos" else \
            fed_cycle(out, g, tau / substeps)
    return out


def build_scale_space(img: np.ndarray, sigma0: float = 1.6, octaves: int = 4,
                      sublevels: int = 4, sigma_cond: float = 1.0,
                      k_percentile: float = 0.7, k_bins: int = 300,
                      k: float | None = None, diffusivity: str = "g2",
                      return_g: bool = False, scheme: str = "aos", substeps: int = 1):
    """Nonlinear scale space (Sec. II-A, Sec. III-A), each level reached by
    one AOS step (Eq. 4) or one FED cycle (Eq. 5), or by ``substeps`` of
    them of equal length (see level_step).

    Returns ``(levels [N][H][W] float64, k)`` and, if ``return_g``, the
    conductivity image of each level's starting image (``g[i]`` drives the
    (first sub-)step into level i; ``g[0]`` is zero).
    """
    f = np.asarray(img, dtype=np.float64)
    sched = level_schedule(sigma0, octaves, sublevels)
    L0 = gaussian_smooth(f, sigma0)
    if k is None:
        k = contrast_factor(L0, sigma_cond, k_percentile, k_bins)
    cond = conductivity_g2 if diffusivity == "g2" else conductivity_g1
    levels = [L0]
    gs = [np.zeros_like(L0)]
    for i in range(1, len(sched)):
        tau = sched[i]["t"] - sched[i - 1]["t"]
        if return_g:
            gs.append(cond(levels[-1], k, sigma_cond))
        levels.append(level_step(levels[-1], k, tau, scheme, substeps, diffusivity, sigma_cond))
    if return_g:
        return np.stack(levels), float(k), np.stack(gs)
    return np.stack(levels), float(k)


# --------------------------------------------------------------------------
# Detector response: Eq. 8 and Sec. II-B
# --------------------------------------------------------------------------
def derivative_step(sigma_n: float) -> int:
    """Scharr step for the normalised scale: round half away from zero, >= 1."""
    return max(1, int(math.floor(sigma_n + 0.5)))


def detector_response(levels: np.ndarray, sigma0: float = 1.6,
                      octaves: int = 4, sublevels: int = 4) -> np.ndarray:
    """Scale-normalised Hessian determinant of every level (Eq. 8)."""
    sched = level_schedule(sigma0, octaves, sublevels)
    out = np.empty_like(np.asarray(levels, dtype=np.float64))
    for lev in sched:
        i = lev["i"]
        sn = lev["sigma"] / 2.0 ** lev["o"]
        s = derivative_step(sn)
        L = np.asarray(levels[i], dtype=np.float64)
        Lx, Ly = scharr_dx(L, s), scharr_dy(L, s)
        Lxx, Lyy, Lxy = scharr_dx(Lx, s), scharr_dy(Ly, s), scharr_dy(Lx, s)
        out[i] = sn * sn * (Lxx * Lyy - Lxy * Lxy)
    return out


def cross_level_radius(sigma: float) -> int:
    """Half-side h of the sigma x sigma window of the exact cross-level
    check: 2h + 1 is the odd side nearest sigma (round half up), at least 3."""
    return max(1, int(math.floor((sigma - 1.0) / 2.0 + 0.5)))


def find_extrema(det: np.ndarray, threshold: float = 0.001, radii=None) -> np.ndarray:
    """3x3x3 maxima above the threshold (Sec. II-B), or with ``radii`` (one
    half-side per level) the exact variant: 3x3 maxima of their own level
    that also exceed levels i-1 and i+1 on the window of half-side radii[i].

    Returns an (n, 4) float64 array with columns level, y, x and response,
    sorted by (level, y, x).
    """
    if radii is not None:
        return _find_extrema_windowed(det, threshold, radii)
    det = np.asarray(det, dtype=np.float64)
    N, H, W = det.shape
    rows = []
    if H < 3 or W < 3:
        return np.zeros((0, 4))
    for i in range(1, N - 1):
        c = det[i, 1:H - 1, 1:W - 1]
        mask = c > threshold
        for dl in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dl == 0 and dy == 0 and dx == 0:
                        continue
                    nb = det[i + dl, 1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
                    mask &= c > nb
        ys, xs = np.nonzero(mask)
        for y, x in zip(ys, xs):
            rows.append((i, y + 1, x + 1, c[y, x]))
    if not rows:
        return np.zeros((0, 4))
    return np.array(sorted(rows), dtype=np.float64)


def _find_extrema_windowed(det, threshold, radii):
    det = np.asarray(det, dtype=np.float64)
    N, H, W = det.shape
    rows = []
    if H < 3 or W < 3:
        return np.zeros((0, 4))
    for i in range(1, N - 1):
        h = int(radii[i])
        # candidates: above the threshold and above the 8 neighbours of level i
        c = det[i, 1:H - 1, 1:W - 1]
        mask = c > threshold
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dy or dx:
                    mask &= c > det[i, 1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
        for y, x in zip(*np.nonzero(mask)):
            y, x = int(y) + 1, int(x) + 1
            v = det[i, y, x]
            y0, y1 = max(0, y - h), min(H, y + h + 1)
            x0, x1 = max(0, x - h), min(W, x + h + 1)
            if np.all(v > det[i - 1, y0:y1, x0:x1]) and np.all(v > det[i + 1, y0:y1, x0:x1]):
                rows.append((i, y, x, v))
    if not rows:
        return np.zeros((0, 4))
    return np.array(rows, dtype=np.float64)


# --------------------------------------------------------------------------
# Description stage (Sec. II-C, Sec. III-C): first derivatives, dominant
# orientation, M-SURF descriptor
# --------------------------------------------------------------------------
def first_derivatives(levels: np.ndarray, sigma0: float = 1.6, octaves: int = 4,
                      sublevels: int = 4):
    """Scale-normalised first derivatives of every level: Lx = sigma_n D_x L,
    Ly = sigma_n D_y L with the detector's Scharr step (Eq. 8)."""
    sched = level_schedule(sigma0, octaves, sublevels)
    lx = np.empty_like(np.asarray(levels, dtype=np.float64))
    ly = np.empty_like(lx)
    for lev in sched:
        i = lev["i"]
        sn = lev["sigma"] / 2.0 ** lev["o"]
        s = derivative_step(sn)
        lx[i] = sn * scharr_dx(levels[i], s)
        ly[i] = sn * scharr_dy(levels[i], s)
    return lx, ly


def _mirror(i, n):
    """Half-sample reflection repeated with period 2n: index into 0..n-1."""
    i = np.mod(i, 2 * n)
    return np.where(i >= n, 2 * n - 1 - i, i)


def bilinear(img: np.ndarray, x, y):
    """Bilinear value of img at real positions (x, y), pixel centres at
    integer coordinates, reflected outside the image."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = x - x0, y - y0
    x0, y0 = x0.astype(np.int64), y0.astype(np.int64)
    xa, xb = _mirror(x0, W), _mirror(x0 + 1, W)
    ya, yb = _mirror(y0, H), _mirror(y0 + 1, H)
    top = (1 - fx) * img[ya, xa] + fx * img[ya, xb]
    bot = (1 - fx) * img[yb, xa] + fx * img[yb, xb]
    return (1 - fy) * top + fy * bot


def orientation_samples():
    """Integer offsets (u, v) with u^2 + v^2 <= 36, row by row (v, then u)."""
    return [(u, v) for v in range(-6, 7) for u in range(-6, 7) if u * u + v * v <= 36]


def dominant_orientation(lx: np.ndarray, ly: np.ndarray, x: float, y: float, s: float):
    """Angle of the longest sum of Gaussian-weighted derivative responses
    over a sliding pi/3 sector (radius 6 s, step s).  Returns (theta, the
    sums' lengths in the order the readings list them)."""
    uv = np.array(orientation_samples(), dtype=np.float64)
    w = np.exp(-(uv[:, 0] ** 2 + uv[:, 1] ** 2) / (2.0 * 2.5 ** 2))
    px, py = x + s * uv[:, 0], y + s * uv[:, 1]
    rx, ry = w * bilinear(lx, px, py), w * bilinear(ly, px, py)
    phi = np.arctan2(ry, rx)
    two_pi, sector = 2.0 * np.pi, np.pi / 3.0
    lengths, sums = [], []
    for k in range(len(phi)):
        d_after = np.mod(phi - phi[k], two_pi)     # phi_j - phi_k in [0, 2 pi)
        d_before = np.mod(phi[k] - phi, two_pi)    # phi_k - phi_j in [0, 2 pi)
        for m in ((d_after > 0.0) & (d_after <= sector), d_before < sector):
            sx, sy = rx[m].sum(), ry[m].sum()
            sums.append((sx, sy))
            lengths.append(math.hypot(sx, sy))
    best = int(np.argmax(lengths))
    return math.atan2(sums[best][1], sums[best][0]), np.array(lengths)


def msurf_descriptor(lx: np.ndarray, ly: np.ndarray, x: float, y: float, s: float,
                     theta: float) -> np.ndarray:
    """64-D M-SURF descriptor of one keypoint (see the readings above)."""
    c, sn = math.cos(theta), math.sin(theta)
    centres = (-7.5, -2.5, 2.5, 7.5)
    out = []
    for b, cv in enumerate(centres):
        for a, cu in enumerate(centres):
            t = np.arange(9, dtype=np.float64) - 4.0
            U, V = np.meshgrid(cu + t, cv + t)
            px = x + s * (U * c - V * sn)
            py = y + s * (U * sn + V * c)
            gx, gy = bilinear(lx, px, py), bilinear(ly, px, py)
            du, dv = gx * c + gy * sn, -gx * sn + gy * c
            w1 = np.exp(-((U - cu) ** 2 + (V - cv) ** 2) / (2.0 * 2.5 ** 2))
            w2 = math.exp(-((a - 1.5) ** 2 + (b - 1.5) ** 2) / (2.0 * 1.5 ** 2))
            out += [w2 * (w1 * du).sum(), w2 * (w1 * dv).sum(),
                    w2 * (w1 * np.abs(du)).sum(), w2 * (w1 * np.abs(dv)).sum()]
    d = np.array(out)
    n = np.linalg.norm(d)
    return d / n if n > 0.0 else d


def describe_keypoints(lx: np.ndarray, ly: np.ndarray, kps: np.ndarray,
                       sigma0: float = 1.6, octaves: int = 4, sublevels: int = 4):
    """Orientation and descriptor of every keypoint; kps rows (level, y, x,
    ...) with real y, x.  Returns (theta (n,), descriptors (n, 64))."""
    sched = level_schedule(sigma0, octaves, sublevels)
    kps = np.asarray(kps, dtype=np.float64).reshape(-1, np.shape(kps)[-1] if len(kps) else 4)
    th, desc = [], []
    for row in kps:
        lev, y, x = int(row[0]), float(row[1]), float(row[2])
        s = sched[lev]["sigma"]
        t, _ = dominant_orientation(lx[lev], ly[lev], x, y, s)
        th.append(t)
        desc.append(msurf_descriptor(lx[lev], ly[lev], x, y, s, t))
    return np.array(th), np.array(desc).reshape(-1, 64)
