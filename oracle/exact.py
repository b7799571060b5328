"""Brute-force kernel filter, Eq. (num) of Section II.  Test infrastructure only.

    g(x) = sum_{y in W_x} w(x-y) k(p(x), p(y)) f(y) / sum_{y in W_x} w(x-y) k(p(x), p(y))

* Spatial kernel (Section IV): Gaussian with covariance sigma_s^2 I on the
  square window |z1|, |z2| <= S, or a box (w == 1) on the same square.
* Range kernel (Section II example, Section IV "covariance theta^2 I"):
  k(t, s) = exp(-|s - t|^2 / (2 sigma_r^2)); sigma_r = inf gives k == 1.
* Borders: the paper is silent; the window is intersected with the image
  domain (zero extension of numerator and denominator alike).
"""
from __future__ import annotations

import numpy as np


def spatial_taps(sigma_s, S, kind="gaussian"):
    """One-dimensional factor w1 of the separable spatial kernel on [-S, S]
    (w(z) = w1(z1) w1(z2)).  Unnormalised: w1(0) = 1."""
    t = np.arange(-S, S + 1, dtype=np.float64)
    if kind == "gaussian":
        return np.exp(-(t * t) / (2.0 * float(sigma_s) ** 2))
    if kind == "box":
        return np.ones_like(t)
    raise ValueError(kind)


def range_kernel_sqdist(d2, sigma_r):
    """k as a function of the squared distance |s - t|^2."""
    if np.isinf(sigma_r):
        return np.ones_like(d2)
    return np.exp(-d2 / (2.0 * float(sigma_r) ** 2))


def patch_guide(f, pr):
    """NLM guide of Section II: the (2pr+1) x (2pr+1) x n patch around each
    pixel, flattened in (dy, dx, channel) row-major order.  Patches near the
    border read a symmetrically padded copy of f (edge sample repeated)."""
    f = np.asarray(f, np.float64)
    H, W, C = f.shape
    fp = np.pad(f, ((pr, pr), (pr, pr), (0, 0)), mode="symmetric")
    T = 2 * pr + 1
    out = np.empty((H, W, T, T, C))
    for dy in range(T):
        for dx in range(T):
            out[:, :, dy, dx, :] = fp[dy:dy + H, dx:dx + W, :]
    return out.reshape(H, W, T * T * C)


def exact_filter(f, p, sigma_s, sigma_r, S, spatial="gaussian", row_block=64):
    """Eq. (num) evaluated by looping over the (2S+1)^2 window offsets.
    ``f`` is [H, W, C], ``p`` is [H, W, D]; returns g as [H, W, C] float64.
    Distances are formed by direct differences."""
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    w1 = spatial_taps(sigma_s, S, spatial)
    num = np.zeros((H, W, C))
    den = np.zeros((H, W))
    for y0 in range(0, H, row_block):
        y1 = min(H, y0 + row_block)
        for dy in range(-S, S + 1):
            # target rows y in [y0, y1) whose neighbour row y+dy lies in the image
            ya, yb = max(y0, -dy), min(y1, H - dy)
            if ya >= yb:
                continue
            for dx in range(-S, S + 1):
                xa, xb = max(0, -dx), min(W, W - dx)
                if xa >= xb:
                    continue
                wsp = w1[dy + S] * w1[dx + S]
                pc = p[ya:yb, xa:xb]
                pn = p[ya + dy:yb + dy, xa + dx:xb + dx]
                diff = pc - pn
                d2 = np.einsum("ijk,ijk->ij", diff, diff)
                wt = wsp * range_kernel_sqdist(d2, sigma_r)
                den[ya:yb, xa:xb] += wt
                num[ya:yb, xa:xb] += wt[:, :, None] * f[ya + dy:yb + dy, xa + dx:xb + dx]
    return num / den[:, :, None]


def exact_filter_at(f, p, sigma_s, sigma_r, S, coords, spatial="gaussian"):
    """Eq. (num) at the listed pixels only; ``coords`` is an [M, 2] array of
    (y, x).  Returns [M, C]."""
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    w1 = spatial_taps(sigma_s, S, spatial)
    out = np.empty((len(coords), C))
    for i, (y, x) in enumerate(np.asarray(coords)):
        ya, yb = max(0, y - S), min(H, y + S + 1)
        xa, xb = max(0, x - S), min(W, x + S + 1)
        wsp = np.outer(w1[ya - y + S:yb - y + S], w1[xa - x + S:xb - x + S])
        diff = p[ya:yb, xa:xb] - p[y, x]
        d2 = np.einsum("ijk,ijk->ij", diff, diff)
        wt = wsp * range_kernel_sqdist(d2, sigma_r)
        out[i] = np.einsum("ij,ijc->c", wt, f[ya:yb, xa:xb]) / wt.sum()
    return out


def psnr(a, b, peak=255.0):
    """Peak signal-to-noise ratio in dB between two images on [0, peak]."""
    mse = np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)
    if mse == 0:
        return np.inf
    return 10.0 * np.log10(peak * peak / mse)
