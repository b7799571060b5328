"""Pins of the float64 gradient reference: it reproduces Algorithm 1's output
(a second formulation of the same K_hat), matches central finite differences,
and obeys exact identities of the filter.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import exact, grad, kmeans, nystrom, seeding
from paper_1901_06112_amd import synth


def _case(h=14, w=12, r=5, seed=21):
    f = synth.rectangles_image(h, w, 5, 20.0, seed=seed).astype(np.float64)
    P = f.reshape(-1, 3)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, seed)], 6)
    G = np.random.default_rng(seed).normal(0, 1, f.shape)
    return f, c, G


def test_torch_formulation_matches_algorithm1():
    f, c, _ = _case()
    g_alg = nystrom.nystrom_filter(f, f, c, 1.5, 30.0, 3)
    g_t = grad.nystrom_torch(torch.tensor(f), torch.tensor(f), torch.tensor(c),
                             torch.tensor(1.5, dtype=torch.float64),
                             torch.tensor(30.0, dtype=torch.float64), 3)
    np.testing.assert_allclose(g_t.numpy(), g_alg, rtol=0, atol=1e-8)


def test_autograd_matches_finite_differences():
    f, c, G = _case()
    ss, sr, S = 1.5, 30.0, 3
    ref = grad.reference_grads(f, f + 0.0, c, ss, sr, S, G)

    def loss(ff, pp, ssv, srv):
        return float((nystrom.nystrom_filter(ff, pp, c, ssv, srv, S) * G).sum())

    fd_sr = grad.central_difference(lambda v: loss(f, f, ss, v), sr)
    fd_ss = grad.central_difference(lambda v: loss(f, f, v, sr), ss)
    assert abs(fd_sr - ref["sigma_r"]) <= 1e-5 * max(1.0, abs(ref["sigma_r"]))
    assert abs(fd_ss - ref["sigma_s"]) <= 1e-5 * max(1.0, abs(ref["sigma_s"]))
    rng = np.random.default_rng(0)
    for _ in range(4):
        y, x, ch = rng.integers(0, f.shape[0]), rng.integers(0, f.shape[1]), rng.integers(0, 3)

        def lf(v):
            ff = f.copy(); ff[y, x, ch] = v
            return loss(ff, f, ss, sr)

        def lp(v):
            pp = f.copy(); pp[y, x, ch] = v
            return loss(f, pp, ss, sr)

        assert abs(grad.central_difference(lf, f[y, x, ch]) - ref["f"][y, x, ch]) <= 1e-6
        assert abs(grad.central_difference(lp, f[y, x, ch]) - ref["p"][y, x, ch]) <= 1e-6


def test_constant_image_has_zero_guide_and_sigma_gradients():
    rng = np.random.default_rng(5)
    f = np.full((12, 11, 3), 90.0)
    p = rng.uniform(0, 255, (12, 11, 3))
    c = p.reshape(-1, 3)[seeding.distinct_indices(132, 5, 5)]
    G = rng.normal(0, 1, f.shape)
    ref = grad.reference_grads(f, p, c, 1.5, 60.0, 3, G)
    assert np.abs(ref["p"]).max() < 1e-10
    assert abs(ref["sigma_r"]) < 1e-9 and abs(ref["sigma_s"]) < 1e-9


def test_shift_equivariance_sum_of_image_gradient():
    # g(f + t) = g(f) + t for a constant shift t, so sum_x dL/df_c = sum_x G_c.
    f, c, G = _case(seed=22)
    ref = grad.reference_grads(f, f, c, 1.5, 30.0, 3, G)
    np.testing.assert_allclose(ref["f"].sum(axis=(0, 1)), G.sum(axis=(0, 1)), rtol=1e-10, atol=1e-10)


def test_single_landmark_large_sigma_r_image_gradient_is_adjoint_blur():
    # r = 1 and sigma_r >> range: K_hat == 1 up to 1e-9, the filter is the
    # normalised blur (w*f)/(w*1), whose adjoint is w * (G / (w*1)).
    f, _, G = _case(seed=23)
    c = np.array([[128.0, 128.0, 128.0]])
    ref = grad.reference_grads(f, f, c, 1.5, 1e7, 3, G)
    w1 = exact.spatial_taps(1.5, 3)
    den = nystrom.conv_zero(np.ones(f.shape[:2]), w1)
    want = nystrom.conv_zero(G / den[:, :, None], w1)
    np.testing.assert_allclose(ref["f"], want, rtol=0, atol=1e-7)
