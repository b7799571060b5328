"""Pins of the brute-force kernel filter (Eq. (num), Section II) and of the
k-means seeding draw, against closed forms, library routines and published
test vectors.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

from oracle import exact, seeding
from paper_1901_06112_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _eval_expr(s):
    s = s.replace("e^-1", "E1").replace("e^-2", "E2").replace("3E2", "3*E2").replace("30E2", "30*E2")
    return eval(s, {"__builtins__": {}}, {"E1": math.exp(-1.0), "E2": math.exp(-2.0)})


def test_hand_examples():
    fx = json.load(open(os.path.join(GOLDEN, "hand_kernel_filter.json")))
    for case in fx["cases"]:
        f = np.array(case["f"], np.float64)
        g = exact.exact_filter(f, f, 1.0 / math.sqrt(2.0), 30.0 / math.sqrt(2.0), 1)
        want = np.array([[_eval_expr(e) for e in row] for row in case["expected_expr"]])
        np.testing.assert_allclose(g[:, :, 0], want, rtol=1e-14, atol=1e-13)


def _normalized_blur_scipy(f, w1):
    num = ndimage.correlate1d(f, w1, axis=0, mode="constant")
    num = ndimage.correlate1d(num, w1, axis=1, mode="constant")
    one = np.ones(f.shape[:2])
    den = ndimage.correlate1d(one, w1, axis=0, mode="constant")
    den = ndimage.correlate1d(den, w1, axis=1, mode="constant")
    return num / den[:, :, None]


@pytest.mark.parametrize("spatial", ["gaussian", "box"])
def test_infinite_sigma_r_is_normalized_blur(spatial):
    f = synth.rectangles_image(23, 31, 5, 10.0, seed=3).astype(np.float64)
    S, ss = 4, 1.7
    g = exact.exact_filter(f, f, ss, np.inf, S, spatial)
    want = _normalized_blur_scipy(f, exact.spatial_taps(ss, S, spatial))
    np.testing.assert_allclose(g, want, rtol=1e-12, atol=1e-10)


def test_constant_guide_is_normalized_blur():
    f = synth.rectangles_image(19, 17, 4, 10.0, seed=4).astype(np.float64)
    p = np.full((19, 17, 3), 42.0)
    g = exact.exact_filter(f, p, 2.0, 5.0, 3)
    want = _normalized_blur_scipy(f, exact.spatial_taps(2.0, 3))
    np.testing.assert_allclose(g, want, rtol=1e-12, atol=1e-10)


def test_constant_image_passes_through():
    rng = np.random.default_rng(0)
    f = np.full((21, 18, 3), 77.0)
    p = rng.uniform(0, 255, (21, 18, 3))
    g = exact.exact_filter(f, p, 3.0, 20.0, 5)
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-12)


def test_tiny_sigma_r_with_distinct_guide_is_identity():
    rng = np.random.default_rng(1)
    p = rng.permutation(np.arange(15 * 13 * 3, dtype=np.float64)).reshape(15, 13, 3)
    f = rng.uniform(0, 255, (15, 13, 2))
    g = exact.exact_filter(f, p, 2.0, 0.05, 3)
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-9)


def test_transpose_and_flip_equivariance():
    f = synth.rectangles_image(17, 26, 6, 15.0, seed=5).astype(np.float64)
    g = exact.exact_filter(f, f, 2.0, 25.0, 4)
    gt = exact.exact_filter(f.transpose(1, 0, 2), f.transpose(1, 0, 2), 2.0, 25.0, 4)
    np.testing.assert_allclose(gt, g.transpose(1, 0, 2), rtol=1e-13, atol=1e-11)
    gf = exact.exact_filter(f[::-1, ::-1], f[::-1, ::-1], 2.0, 25.0, 4)
    np.testing.assert_allclose(gf, g[::-1, ::-1], rtol=1e-13, atol=1e-11)


def test_pointwise_matches_full():
    f = synth.rectangles_image(20, 24, 6, 15.0, seed=6).astype(np.float64)
    g = exact.exact_filter(f, f, 2.0, 25.0, 5)
    coords = np.array([[0, 0], [19, 23], [7, 11], [0, 12], [13, 0]])
    gp = exact.exact_filter_at(f, f, 2.0, 25.0, 5, coords)
    np.testing.assert_allclose(gp, g[coords[:, 0], coords[:, 1]], rtol=1e-13, atol=1e-11)


def test_patch_guide_layout_and_border():
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, (6, 7, 3))
    P = exact.patch_guide(f, 1)
    assert P.shape == (6, 7, 27)
    # interior pixel: entries in (dy, dx, c) order
    y, x = 3, 4
    want = np.concatenate([f[y + dy, x + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    np.testing.assert_array_equal(P[y, x], want)
    # corner: row/column -1 repeats row/column 0
    want0 = np.concatenate([f[max(dy, 0), max(dx, 0)] for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    np.testing.assert_array_equal(P[0, 0], want0)


def test_splitmix64_published_vector():
    fx = json.load(open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")))
    g = seeding.SplitMix64(fx["seed"])
    assert [g.next() for _ in range(5)] == [int(v) for v in fx["outputs"]]


def test_distinct_indices():
    for n, r, s in [(10, 10, 0), (1000, 37, 5), (4 * 10**6, 64, 9), (1, 1, 3)]:
        idx = seeding.distinct_indices(n, r, s)
        assert len(set(idx.tolist())) == r
        assert idx.min() >= 0 and idx.max() < n
    perm = seeding.distinct_indices(50, 50, 11)
    assert sorted(perm.tolist()) == list(range(50))
    with pytest.raises(ValueError):
        seeding.distinct_indices(5, 6, 0)


def test_distinct_indices_hand_derived_draw():
    """The draw order j = i + next() mod (N - i), with the swaps of a partial
    Fisher-Yates shuffle, against draws derived by hand from the published
    SplitMix64 outputs (tests/golden/fisher_yates_seed1234567.json); the
    N = 10 case reuses a position that an earlier step moved."""
    fx = json.load(open(os.path.join(GOLDEN, "fisher_yates_seed1234567.json")))
    for case in fx["cases"]:
        got = seeding.distinct_indices(case["N"], case["r"], fx["seed"])
        assert got.tolist() == case["idx"], case["N"]


def test_psnr_known_values():
    """PSNR = 10 log10(peak^2 / MSE): values fixed by the definition, at peaks
    1 and 255."""
    a = np.zeros((8, 8, 3))
    # peak 1, every error 0.1: MSE 0.01 -> exactly 20 dB
    assert exact.psnr(a + 0.1, a, peak=1.0) == pytest.approx(20.0, abs=1e-12)
    # peak 255, every error 25.5 (a tenth of the peak): 20 dB
    assert exact.psnr(a + 25.5, a, peak=255.0) == pytest.approx(20.0, abs=1e-12)
    # every error 1 on the 0..255 scale: 20 log10(255) = 48.1308036... dB
    assert exact.psnr(a + 1.0, a) == pytest.approx(48.13080360867910, abs=1e-10)
    # errors of opposite sign count alike; half the pixels wrong by 2:
    # MSE 2 -> 48.1308 - 10 log10(2) = 45.1205 dB
    b = a.copy()
    b[::2] += 2.0
    b[1::2] -= 0.0
    assert exact.psnr(b, a) == pytest.approx(45.12050365203929, abs=1e-10)
    c = a.copy()
    c[::2] -= 2.0
    assert exact.psnr(c, a) == exact.psnr(b, a)
    # identical images: infinite
    assert exact.psnr(a, a) == np.inf
    # symmetric in its arguments and invariant to a common scale of data and peak
    rng = np.random.default_rng(4)
    x, y = rng.uniform(0, 255, (2, 16, 16, 3))
    assert exact.psnr(x, y) == pytest.approx(exact.psnr(y, x), abs=1e-12)
    assert exact.psnr(x / 255.0, y / 255.0, peak=1.0) == pytest.approx(exact.psnr(x, y), abs=1e-9)
