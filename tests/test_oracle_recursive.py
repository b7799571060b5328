"""Pins of the recursive Gaussian oracle (Young and van Vliet's IIR filter,
the O(1) Gaussian of Section IV) and of Algorithm 1 with it.  CPU only."""

import numpy as np
import pytest

from oracle import exact, nystrom, recursive, seeding
from paper_1901_06112_amd import synth

SIGMAS = [0.5, 1.0, 2.0, 2.5, 3.0, 5.0, 8.0, 12.0, 20.0]


def _pole_form(q):
    """b0..b3 rebuilt from Young and van Vliet's s-plane poles (m0 real,
    m1 +- i m2) mapped by the scale q: b0 = (m0 + q)(m1^2 + m2^2 + 2 m1 q + q^2),
    b1 = q (2 m0 m1 + m1^2 + m2^2 + (2 m0 + 4 m1) q + 3 q^2),
    b2 = -q^2 (m0 + 2 m1 + 3 q), b3 = q^3 (common factor dropped)."""
    m0, m1, m2 = 1.16680, 1.10783, 1.40586
    b0 = (m0 + q) * (m1 * m1 + m2 * m2 + 2 * m1 * q + q * q)
    b1 = q * (2 * m0 * m1 + m1 * m1 + m2 * m2 + (2 * m0 + 4 * m1) * q + 3 * q * q)
    b2 = -q * q * (m0 + 2 * m1 + 3 * q)
    b3 = q ** 3
    return b1 / b0, b2 / b0, b3 / b0


@pytest.mark.parametrize("q", [0.1, 0.5, 1.0, 2.0, 4.0, 9.0, 20.0])
def test_polynomial_coefficients_match_the_pole_form(q):
    # the published polynomials are the pole form with six-digit coefficients
    a1, a2, a3, B = recursive.yv_coefficients(q)
    np.testing.assert_allclose([a1, a2, a3], _pole_form(q), rtol=2e-5, atol=0)
    assert abs(B + a1 + a2 + a3 - 1.0) < 1e-15


def test_scale_branches_meet_and_grow():
    qs = [recursive.scale_for_sigma(s) for s in np.linspace(0.5, 30, 300)]
    assert all(b > a for a, b in zip(qs, qs[1:]))
    assert recursive.scale_for_sigma(0.5) > 0
    with pytest.raises(ValueError):
        recursive.scale_for_sigma(0.49)


@pytest.mark.parametrize("sigma", SIGMAS)
def test_impulse_response_sum_symmetry_and_variance(sigma):
    half = recursive.padding(sigma) + int(10 * sigma)
    h = recursive.impulse_response(sigma, half)
    n = np.arange(-half, half + 1)
    assert abs(h.sum() - 1.0) < 1e-12                       # unit DC gain
    assert np.abs(h - h[::-1]).max() < 1e-13 * h.max()      # zero phase
    assert h.min() > -1e-13 * h.max()                       # no lobes beyond rounding
    # second moment of the computed response against the closed form
    var = (h * n * n).sum()
    q = recursive.scale_for_sigma(sigma)
    assert abs(var - recursive.response_variance(q)) < 1e-10 * var
    # the fit is for shape: about 10% wider than sigma, never narrower
    assert sigma ** 2 < var < 1.6 * sigma ** 2


# largest |h - g_sigma| / max g_sigma of the fit, from the measured responses
# (7.6% at 0.5, 9.4% at 1, 5.2% at 2, 3.2% at 5, 1.5% at 20) with ~15% margin
SHAPE_TOL = {0.5: 0.088, 1.0: 0.108, 2.0: 0.060, 2.5: 0.063, 3.0: 0.046, 5.0: 0.037,
             8.0: 0.029, 12.0: 0.023, 20.0: 0.018}


@pytest.mark.parametrize("sigma", SIGMAS)
def test_impulse_response_approximates_the_sampled_gaussian(sigma):
    half = recursive.padding(sigma) + int(10 * sigma)
    h = recursive.impulse_response(sigma, half)
    n = np.arange(-half, half + 1)
    g = np.exp(-n * n / (2.0 * sigma * sigma))
    g /= g.sum()
    err = np.abs(h - g).max() / g.max()
    assert err < SHAPE_TOL[sigma]
    # and a wrong scale (q off by 10%) would be much further away for sigma >= 2
    if sigma >= 2.0:
        q = recursive.scale_for_sigma(sigma)
        assert abs(recursive.response_variance(1.1 * q) - recursive.response_variance(q)) > 0.15 * sigma ** 2


@pytest.mark.parametrize("sigma,n", [(1.5, 23), (4.0, 31), (9.0, 12), (3.0, 1)])
def test_border_rule_is_convolution_with_the_zero_extended_line(sigma, n):
    # brute force: the output is sum_j h[i - j] x[j] over the line only
    rng = np.random.default_rng(int(10 * sigma) + n)
    x = rng.uniform(-5, 5, n)
    half = recursive.padding(sigma) + n
    h = recursive.impulse_response(sigma, half)
    want = np.array([sum(h[half + i - j] * x[j] for j in range(n)) for i in range(n)])
    np.testing.assert_allclose(recursive.recursive_gauss_1d(x, sigma), want, rtol=0, atol=1e-13)


def test_constant_line_interior_and_2d_separability():
    y = recursive.recursive_gauss_1d(np.full(600, 3.0), 5.0)
    np.testing.assert_allclose(y[250:350], 3.0, rtol=0, atol=1e-12)
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 1, (17, 26, 2))
    rows_first = recursive.recursive_gauss_2d(img, 2.2)
    cols_first = recursive.recursive_gauss_1d(recursive.recursive_gauss_1d(img, 2.2, axis=0), 2.2, axis=1)
    np.testing.assert_allclose(rows_first, cols_first, rtol=0, atol=1e-14)


# ----------------------------------------------- Algorithm 1 with the IIR

def _brute_force_recursive_filter(f, p, sigma_s, sigma_r):
    """Eq. (num) with the spatial weight h(y1 - x1) h(y2 - x2) over the whole
    image (the recursive Gaussian's 2-D response) and the exact range kernel."""
    H, W, C = f.shape
    half = recursive.padding(sigma_s) + max(H, W)
    h = recursive.impulse_response(sigma_s, half)
    P = p.reshape(-1, p.shape[2])
    K = exact.range_kernel_sqdist(nystrom.sqdist(P, P), sigma_r)
    ys, xs = np.divmod(np.arange(H * W), W)
    Ws = h[half + ys[:, None] - ys[None, :]] * h[half + xs[:, None] - xs[None, :]]
    wt = Ws * K
    return ((wt @ f.reshape(-1, C)) / wt.sum(1)[:, None]).reshape(H, W, C)


def test_nystrom_recursive_exact_with_all_distinct_guide_values():
    rng = np.random.default_rng(11)
    cols = rng.uniform(0, 255, (6, 3))
    lab = rng.integers(0, 6, (9, 11))
    f = cols[lab]
    used = np.unique(f.reshape(-1, 3), axis=0)
    want = _brute_force_recursive_filter(f, f, 2.0, 70.0)
    got = nystrom.nystrom_filter(f, f, used, 2.0, 70.0, 0, spatial="recursive")
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-8)


def test_nystrom_recursive_constant_image_and_infinite_sigma_r():
    rng = np.random.default_rng(12)
    p = rng.uniform(0, 255, (14, 13, 3))
    c = p.reshape(-1, 3)[seeding.distinct_indices(14 * 13, 7, 4)]
    g = nystrom.nystrom_filter(np.full((14, 13, 3), 42.0), p, c, 3.0, 30.0, 0, spatial="recursive")
    np.testing.assert_allclose(g, 42.0, rtol=0, atol=1e-9)
    f = synth.rectangles_image(14, 13, 4, 10.0, seed=3).astype(np.float64)
    g = nystrom.nystrom_filter(f, f, c, 3.0, 1e7, 0, spatial="recursive")
    num = recursive.recursive_gauss_2d(f, 3.0)
    den = recursive.recursive_gauss_2d(np.ones((14, 13)), 3.0)
    np.testing.assert_allclose(g, num / den[:, :, None], rtol=0, atol=1e-6)
