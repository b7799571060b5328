"""Pins of the PCA patch-guide oracle (PCA-NLM, Section IV) against closed
forms and invariants.  CPU only."""
import numpy as np

from oracle import exact, pca, seeding
from paper_1901_06112_amd import synth


def _img(h, w, c, seed):
    """Noisy rectangles, first c of its 3 channels."""
    return np.ascontiguousarray(synth.rectangles_image(h, w, 8, 20.0, seed=seed)[:, :, :c]).astype(np.float64)


def test_basis_orthonormal_descending_signed():
    f = _img(30, 34, 3, 1)
    mu, V, lam = pca.patch_pca(f, 1, 10)
    assert V.shape == (27, 10) and mu.shape == (27,)
    np.testing.assert_allclose(V.T @ V, np.eye(10), atol=1e-12)
    assert np.all(np.diff(lam) <= 0) and lam[-1] > 0
    for k in range(10):
        j = int(np.argmax(np.abs(V[:, k])))
        assert V[j, k] > 0


def test_projected_sample_moments_are_the_eigenvalues():
    """The projections of the sample have zero mean and covariance diag(lam):
    V holds eigenvectors of the sample covariance with eigenvalues lam."""
    f = _img(40, 37, 3, 2)
    mu, V, lam = pca.patch_pca(f, 1, 8)
    P = exact.patch_guide(f, 1).reshape(-1, 27)
    G = (P - mu) @ V
    np.testing.assert_allclose(G.mean(axis=0), 0.0, atol=1e-9 * np.sqrt(lam[0]))
    cov_g = G.T @ G / G.shape[0]
    np.testing.assert_allclose(cov_g, np.diag(lam), atol=1e-10 * lam[0])
    # and no unit direction holds more variance than the first one
    rng = np.random.default_rng(0)
    X = P - P.mean(axis=0)
    for _ in range(20):
        v = rng.normal(size=27)
        v /= np.linalg.norm(v)
        assert np.mean((X @ v) ** 2) <= lam[0] * (1 + 1e-12)


def test_full_dimension_preserves_distances():
    """dim = D is a rotation of the centred patches: every pairwise distance
    between guide values equals the distance between the patches."""
    f = _img(9, 8, 2, 3)
    g, lam = pca.pca_guide(f, 1, 18)
    P = exact.patch_guide(f, 1).reshape(-1, 18)
    G = g.reshape(-1, 18)
    dP = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    dG = ((G[:, None, :] - G[None, :, :]) ** 2).sum(-1)
    np.testing.assert_allclose(dG, dP, rtol=1e-10, atol=1e-8)


def test_matches_svd_of_the_centred_sample():
    f = _img(33, 31, 3, 4)
    mu, V, lam = pca.patch_pca(f, 1, 6)
    P = exact.patch_guide(f, 1).reshape(-1, 27)
    X = P - P.mean(axis=0)
    _, s, Vt = np.linalg.svd(X, full_matrices=False)
    np.testing.assert_allclose(lam, s[:6] ** 2 / X.shape[0], rtol=1e-10)
    for k in range(6):
        assert abs(abs(Vt[k] @ V[:, k]) - 1.0) < 1e-9


def test_pixels_on_a_line_give_a_rank_one_basis():
    """pr = 0: patches are the pixel values.  Values m + t(x) d on a line give
    v_1 = d / |d| (positive largest entry), lam_1 = var(t) |d|^2 and nothing
    else; the guide is (t - mean t) |d|."""
    rng = np.random.default_rng(5)
    t = rng.uniform(-3, 3, (20, 25))
    m, d = np.array([40.0, 80.0, 120.0]), np.array([2.0, -5.0, 1.0])
    f = m + t[:, :, None] * d
    mu, V, lam = pca.patch_pca(f, 0, 3)
    nd = np.linalg.norm(d)
    np.testing.assert_allclose(V[:, 0], -d / nd, atol=1e-12)   # largest entry (-5) made positive
    np.testing.assert_allclose(lam[0], t.var() * nd * nd, rtol=1e-12)
    assert abs(lam[1]) < 1e-12 * lam[0] and abs(lam[2]) < 1e-12 * lam[0]
    g, _ = pca.pca_guide(f, 0, 1)
    np.testing.assert_allclose(g[:, :, 0], -(t - t.mean()) * nd, atol=1e-10)


def test_large_images_use_the_seeded_sample():
    """N > 65536: the basis comes from the patches of the seeded draw."""
    f = _img(260, 256, 1, 6)
    idx = pca.sample_indices(f.shape[0] * f.shape[1], 11)
    assert len(idx) == pca.SAMPLE_MAX and len(np.unique(idx)) == pca.SAMPLE_MAX
    np.testing.assert_array_equal(idx, seeding.distinct_indices(f.shape[0] * f.shape[1], pca.SAMPLE_MAX, 11))
    mu, V, lam = pca.patch_pca(f, 1, 3, seed=11)
    P = exact.patch_guide(f, 1).reshape(-1, 9)
    np.testing.assert_allclose(mu, P[idx].mean(axis=0), rtol=1e-13)
