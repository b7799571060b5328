"""Seeded synthetic workloads for Nystrom kernel filtering.

This module only draws test images. It contains none of the filter's
arithmetic and is the single input source shared by the oracle-based tests,
the GPU parity tests and the benchmark.

The paper evaluates on colour photographs and a hyperspectral scene
(Section IV); those datasets are not available, so each workload below is a
synthetic stand-in with the same shape, value range and kind of structure:
piecewise-constant colour regions plus Gaussian noise for colour BLF/NLM,
smooth fields plus polygons for the large colour case, and linear mixtures of
smooth positive spectra for the hyperspectral case.  All images are clipped to
[0, R] as the problem statement in Section II requires (R = 255 for colour,
R = 1 for hyperspectral).

Every generator takes an explicit ``seed`` and uses numpy's PCG64.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "rectangles_image",
    "perlin_polygons_image",
    "hyperspectral_cube",
    "batch_sizes",
    "workload",
    "WORKLOADS",
]


def rectangles_image(h, w, n_rect=12, noise=20.0, seed=0, dtype=np.float32):
    """Piecewise-constant colour image: a uniform background and ``n_rect``
    axis-aligned rectangles painted in order, then i.i.d. N(0, noise^2), clipped
    to [0, 255].  Returns ``[h, w, 3]``."""
    rng = np.random.default_rng(seed)
    img = np.empty((h, w, 3), np.float64)
    img[:] = rng.uniform(0.0, 255.0, 3)
    for _ in range(n_rect):
        ys = np.sort(rng.integers(0, h + 1, 2))
        xs = np.sort(rng.integers(0, w + 1, 2))
        col = rng.uniform(0.0, 255.0, 3)
        img[ys[0]:ys[1], xs[0]:xs[1]] = col
    if noise > 0:
        img += rng.normal(0.0, noise, img.shape)
    np.clip(img, 0.0, 255.0, out=img)
    return img.astype(dtype)


def _value_noise(h, w, rng, spacings=(256, 128, 64, 32)):
    """Sum of octaves of bicubically upsampled uniform grids, per channel."""
    acc = np.zeros((h, w, 3), np.float64)
    amp = 1.0
    for s in spacings:
        gh, gw = h // s + 4, w // s + 4
        grid = rng.uniform(0.0, 1.0, (gh, gw, 3))
        for c in range(3):
            up = ndimage.zoom(grid[:, :, c], s, order=3, mode="nearest", grid_mode=True)
            acc[:, :, c] += amp * up[s:s + h, s:s + w]
        amp *= 0.5
    lo = acc.min(axis=(0, 1), keepdims=True)
    hi = acc.max(axis=(0, 1), keepdims=True)
    return 255.0 * (acc - lo) / np.maximum(hi - lo, 1e-12)


def _paint_convex_polygon(img, rng):
    h, w, _ = img.shape
    nv = int(rng.integers(3, 9))
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, nv))
    rad = rng.uniform(20.0, 300.0)
    cy, cx = rng.uniform(0.0, h), rng.uniform(0.0, w)
    col = rng.uniform(0.0, 255.0, 3)
    vy = cy + rad * np.sin(ang)
    vx = cx + rad * np.cos(ang)
    y0, y1 = max(int(np.floor(vy.min())), 0), min(int(np.ceil(vy.max())) + 1, h)
    x0, x1 = max(int(np.floor(vx.min())), 0), min(int(np.ceil(vx.max())) + 1, w)
    if y0 >= y1 or x0 >= x1:
        return
    yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    inside = np.ones(yy.shape, bool)
    # vertices lie on a circle in angular order, so the polygon is convex and
    # counter-clockwise in (x, y): inside means left of every edge.
    for i in range(nv):
        ax, ay = vx[i], vy[i]
        bx, by = vx[(i + 1) % nv], vy[(i + 1) % nv]
        inside &= (bx - ax) * (yy - ay) - (by - ay) * (xx - ax) >= 0.0
    img[y0:y1, x0:x1][inside] = col


def perlin_polygons_image(h, w, n_poly=30, noise=25.0, seed=0, dtype=np.float32):
    """Smooth 4-octave value-noise colour field, 30 random convex polygons of
    uniform colour painted in order, N(0, noise^2), clipped to [0, 255]."""
    rng = np.random.default_rng(seed)
    img = _value_noise(h, w, rng)
    for _ in range(n_poly):
        _paint_convex_polygon(img, rng)
    if noise > 0:
        img += rng.normal(0.0, noise, img.shape)
    np.clip(img, 0.0, 255.0, out=img)
    return img.astype(dtype)


def hyperspectral_cube(h, w, bands=128, n_end=8, noise=0.02, seed=0, dtype=np.float32):
    """Linear mixture of ``n_end`` smooth positive endmember spectra with
    spatially smoothed Dirichlet(0.5) abundances, plus N(0, noise^2), clipped to
    [0, 1].  Returns ``[h, w, bands]``."""
    rng = np.random.default_rng(seed)
    t = np.arange(bands, dtype=np.float64)
    ends = np.empty((n_end, bands))
    for e in range(n_end):
        s = np.full(bands, 0.05)
        for _ in range(3):
            mu = rng.uniform(0.0, bands - 1.0)
            wd = rng.uniform(8.0, 40.0)
            ht = rng.uniform(0.2, 1.0)
            s += ht * np.exp(-0.5 * ((t - mu) / wd) ** 2)
        ends[e] = s / s.max()
    ab = rng.dirichlet(0.5 * np.ones(n_end), size=(h, w))
    for e in range(n_end):
        ab[:, :, e] = ndimage.gaussian_filter(ab[:, :, e], 8.0, mode="reflect")
    ab /= ab.sum(axis=2, keepdims=True)
    cube = ab.reshape(-1, n_end) @ ends
    cube = cube.reshape(h, w, bands)
    if noise > 0:
        cube += rng.normal(0.0, noise, cube.shape)
    np.clip(cube, 0.0, 1.0, out=cube)
    return cube.astype(dtype)


def batch_sizes(n=8, lo=384, hi=1024, seed=1050):
    """Image sizes of the ragged differentiation batch: i.i.d. uniform
    integers in [lo, hi] per side."""
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))) for _ in range(n)]


# Parameters of the five workloads.  ``S`` is the window radius (window width
# 2S+1); ``sigma_r`` is the range-kernel width in exp(-|s-t|^2 / (2 sigma_r^2)).
WORKLOADS = {
    "color_blf_256": dict(H=256, W=256, C=3, guide="self", sigma_s=3.0, S=9, sigma_r=30.0,
                          r=16, iters=10, spatial="gaussian", seed=1001, landmark_seed=1),
    "color_blf_2048": dict(H=2048, W=2048, C=3, guide="self", sigma_s=5.0, S=15, sigma_r=40.0,
                           r=32, iters=15, spatial="gaussian", seed=1002, landmark_seed=2),
    "hyperspectral_512x128": dict(H=512, W=512, C=128, guide="self", sigma_s=4.0, S=12,
                                  sigma_r=0.3, r=64, iters=10, spatial="gaussian", seed=1003,
                                  landmark_seed=3),
    "color_nlm_1024": dict(H=1024, W=1024, C=3, guide="patch", patch_radius=3, sigma_s=10.0,
                           S=10, sigma_r=10.0 * np.sqrt(147.0), r=128, iters=10, spatial="box",
                           seed=1004, landmark_seed=4),
    # PCA-NLM: the NLM image, patches reduced by PCA to 25 dimensions, m0 = 31
    # landmarks, theta = 3 x the noise level (Section IV)
    "color_pca_nlm_1024": dict(H=1024, W=1024, C=3, guide="pca", patch_radius=3, pca_dim=25, sigma_s=10.0,
                               S=10, sigma_r=90.0, r=31, iters=10, spatial="box", seed=1004,
                               landmark_seed=4),
    "diff_batch8": dict(C=3, guide="self", sigma_s=3.0, S=9, sigma_r=30.0, r=32, iters=10,
                        spatial="gaussian", seed=1050, landmark_seed=5, n_images=8),
}


def workload(name, h=None, w=None, seed=None):
    """Image (and guide, when explicit) of a named workload, optionally at a
    reduced size ``h x w`` for fast tests.  Returns ``(f, params)``; the guide
    is ``f`` itself for ``guide == 'self'`` and the 7x7x3 patch vector of ``f``
    for ``guide == 'patch'`` (formed by the filter, not here)."""
    prm = dict(WORKLOADS[name])
    H = prm.get("H") if h is None else h
    W = prm.get("W") if w is None else w
    sd = prm["seed"] if seed is None else seed
    if name == "color_blf_256":
        f = rectangles_image(H, W, 12, 20.0, sd)
    elif name == "color_blf_2048":
        f = perlin_polygons_image(H, W, 30, 25.0, sd)
    elif name == "hyperspectral_512x128":
        f = hyperspectral_cube(H, W, prm["C"], 8, 0.02, sd)
    elif name in ("color_nlm_1024", "color_pca_nlm_1024"):
        f = rectangles_image(H, W, 12, 30.0, sd)
    elif name == "diff_batch8":
        f = rectangles_image(H, W, 12, 20.0, sd)
    else:
        raise KeyError(name)
    prm["H"], prm["W"] = H, W
    return f, prm
