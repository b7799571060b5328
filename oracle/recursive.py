"""Recursive (IIR) Gaussian spatial filter.  Test infrastructure only.

Section IV evaluates the Gaussian-window convolutions of Eqs. (finalnum) and
(finalden) with Young and van Vliet's O(1) recursive Gaussian (Signal
Processing 44, 1995) instead of the truncated window.  The filter is a causal
third-order recursion followed by the same recursion run backwards:

    w[n] = B x[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3]      (forward)
    y[n] = B w[n] + a1 y[n+1] + a2 y[n+2] + a3 y[n+3]      (backward)

with a_i = b_i / b0 and B = 1 - a1 - a2 - a3 (unit DC gain), where b0..b3 are
Young and van Vliet's polynomials in the scale q, and q is their fit to the
Gaussian's sigma (sigma >= 0.5).  The cascade's impulse response h is
symmetric, sums to one, has a closed-form variance (about 10% above sigma^2:
the fit matches the Gaussian's shape, not its second moment) and differs
from the sampled Gaussian by a few percent of its peak.

Readings where the paper is silent:
* border: the image is extended by zeros, in numerator and denominator alike,
  as for the truncated window.  The filtered line is h convolved with the
  zero-extended line; here that is computed by running the cascade over the
  line padded with enough zeros on both sides that the response has decayed
  below FP64 resolution, then cropping.
* 2-D: rows then columns (the 2-D filter is separable, w(z) = w1(z1) w1(z2)).
"""
from __future__ import annotations

import math

import numpy as np


def yv_coefficients(q):
    """(a1, a2, a3, B) of the recursion for scale q: Young and van Vliet's
    polynomials b0..b3 in q, normalised by b0."""
    b0 = 1.57825 + 2.44413 * q + 1.4281 * q ** 2 + 0.422205 * q ** 3
    b1 = 2.44413 * q + 2.85619 * q ** 2 + 1.26661 * q ** 3
    b2 = -(1.4281 * q ** 2 + 1.26661 * q ** 3)
    b3 = 0.422205 * q ** 3
    a = (b1 / b0, b2 / b0, b3 / b0)
    return a[0], a[1], a[2], 1.0 - a[0] - a[1] - a[2]


def response_variance(q):
    """Variance of the forward-backward cascade's impulse response.

    The causal part H(z) = B / (1 - sum_j a_j z^-j) has unit DC gain; its
    cumulant generating function is log B - log(1 - sum_j a_j e^{j t}), whose
    second derivative at t = 0 is its variance,
        sum_j j^2 a_j / B + (sum_j j a_j / B)^2.
    The backward pass is its mirror image, so the cascade has twice that."""
    a1, a2, a3, B = yv_coefficients(q)
    m1 = (1 * a1 + 2 * a2 + 3 * a3) / B
    m2 = (1 * a1 + 4 * a2 + 9 * a3) / B
    return 2.0 * (m2 + m1 * m1)


def scale_for_sigma(sigma):
    """Young and van Vliet's q for a Gaussian of width sigma >= 0.5: linear
    in sigma from 2.5 on, a square-root law below."""
    sigma = float(sigma)
    if sigma < 0.5:
        raise ValueError("the recursive Gaussian needs sigma >= 0.5")
    if sigma >= 2.5:
        return 0.98711 * sigma - 0.96330
    return 3.97156 - 4.14554 * math.sqrt(1.0 - 0.26891 * sigma)


def padding(sigma):
    """Zeros added on each side of a line: the slowest pole p of the causal
    recursion decays below 1e-20 over this many samples."""
    a1, a2, a3, _ = yv_coefficients(scale_for_sigma(sigma))
    p = np.abs(np.roots([1.0, -a1, -a2, -a3])).max()
    return int(math.ceil(math.log(1e-20) / math.log(p))) + 8


def recursive_gauss_1d(x, sigma, axis=-1):
    """The cascade along ``axis`` of ``x`` (any shape), zero-extended."""
    x = np.moveaxis(np.asarray(x, np.float64), axis, -1)
    a1, a2, a3, B = yv_coefficients(scale_for_sigma(sigma))
    L = padding(sigma)
    n = x.shape[-1]
    xp = np.zeros(x.shape[:-1] + (n + 2 * L,))
    xp[..., L:L + n] = x
    m = xp.shape[-1]
    w = np.zeros(x.shape[:-1] + (m + 3,))          # w[..., i + 3] holds w[i]
    for i in range(m):
        w[..., i + 3] = B * xp[..., i] + a1 * w[..., i + 2] + a2 * w[..., i + 1] + a3 * w[..., i]
    y = np.zeros(x.shape[:-1] + (m + 3,))          # y[..., i] holds y[i]
    for i in range(m - 1, -1, -1):
        y[..., i] = B * w[..., i + 3] + a1 * y[..., i + 1] + a2 * y[..., i + 2] + a3 * y[..., i + 3]
    return np.moveaxis(y[..., L:L + n], -1, axis)


def recursive_gauss_2d(img, sigma):
    """Rows then columns of ``img`` [H, W] or [H, W, ...]."""
    return recursive_gauss_1d(recursive_gauss_1d(img, sigma, axis=1), sigma, axis=0)


def impulse_response(sigma, half):
    """h[-half..half]: the cascade applied to a unit impulse in the middle of
    a zero line of length 2 half + 1."""
    e = np.zeros(2 * half + 1)
    e[half] = 1.0
    return recursive_gauss_1d(e, sigma)
