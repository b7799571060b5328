"""Pins of the k-means oracle and of Algorithm 1 (Section III) against what
the paper and the mathematics fix.  CPU only."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import exact, kmeans, nystrom, seeding
from paper_1901_06112_amd import synth


# ----------------------------------------------------------------- k-means

def test_lloyd_objective_non_increasing_and_fixed_point():
    f = synth.rectangles_image(40, 36, 8, 20.0, seed=7)
    P = f.reshape(-1, 3).astype(np.float64)
    c0 = P[seeding.distinct_indices(P.shape[0], 9, 3)]
    c, lab, errs = kmeans.lloyd(P, c0, 25)
    assert all(b <= a * (1 + 1e-14) for a, b in zip(errs, errs[1:]))
    # after convergence every non-empty centroid is the mean of its members
    lab2, _ = kmeans.assign(P, c)
    c2, _, cnt = kmeans.update(P, lab2, c)
    if np.array_equal(lab2, lab):
        np.testing.assert_allclose(c2, c, rtol=1e-13, atol=1e-10)


def test_lloyd_recovers_separated_clusters():
    rng = np.random.default_rng(0)
    centers = np.array([[0, 0, 0], [100, 0, 0], [0, 100, 0], [0, 0, 100]], np.float64)
    P = np.concatenate([c + rng.normal(0, 1.0, (200, 3)) for c in centers])
    c0 = P[[0, 200, 400, 600]]
    c, lab, _ = kmeans.lloyd(P, c0, 5)
    for k in range(4):
        np.testing.assert_allclose(c[k], P[200 * k:200 * (k + 1)].mean(0), rtol=0, atol=1e-12)


def test_assign_ties_go_to_lowest_index_and_empty_keeps():
    P = np.array([[0.0], [2.0]])
    c = np.array([[1.0], [1.0], [50.0]])
    lab, _ = kmeans.assign(P, c)
    assert lab.tolist() == [0, 0]
    c2, _, cnt = kmeans.update(P, lab, c)
    assert cnt.tolist() == [2, 0, 0]
    np.testing.assert_array_equal(c2[1:], c[1:])


# ------------------------------------------------------------- Nystrom

def _few_colour_image(h, w, seed, ncol=5):
    rng = np.random.default_rng(seed)
    cols = rng.uniform(0, 255, (ncol, 3))
    lab = np.zeros((h, w), int)
    for i in range(1, ncol):
        y0, x0 = rng.integers(0, h - 2), rng.integers(0, w - 2)
        lab[y0:y0 + rng.integers(2, h), x0:x0 + rng.integers(2, w)] = i
    return cols[lab], cols


def test_exact_when_landmarks_are_all_distinct_guide_values():
    f, cols = _few_colour_image(24, 21, 1)
    used = np.unique(f.reshape(-1, 3), axis=0)
    g = exact.exact_filter(f, f, 2.0, 60.0, 4)
    gh = nystrom.nystrom_filter(f, f, used, 2.0, 60.0, 4)
    np.testing.assert_allclose(gh, g, rtol=0, atol=1e-9)


def test_constant_image_passes_through():
    rng = np.random.default_rng(3)
    f = np.full((22, 19, 3), 77.0)
    p = rng.uniform(0, 255, (22, 19, 3))
    c = p.reshape(-1, 3)[seeding.distinct_indices(22 * 19, 8, 1)]
    gh = nystrom.nystrom_filter(f, p, c, 2.0, 40.0, 4)
    np.testing.assert_allclose(gh, f, rtol=0, atol=1e-9)


def test_huge_sigma_r_is_normalized_blur():
    f = synth.rectangles_image(25, 30, 6, 15.0, seed=8).astype(np.float64)
    c = f.reshape(-1, 3)[seeding.distinct_indices(25 * 30, 6, 2)]
    alpha, _ = nystrom.landmark_eig(c, 1e7)
    assert len(alpha) == 1
    gh = nystrom.nystrom_filter(f, f, c, 2.5, 1e7, 5)
    w1 = exact.spatial_taps(2.5, 5)
    num = ndimage.correlate1d(ndimage.correlate1d(f, w1, axis=0, mode="constant"), w1, axis=1,
                              mode="constant")
    den = ndimage.correlate1d(ndimage.correlate1d(np.ones((25, 30)), w1, axis=0, mode="constant"),
                              w1, axis=1, mode="constant")
    np.testing.assert_allclose(gh, num / den[:, :, None], rtol=0, atol=1e-6)


def test_khat_closed_form_and_psd_gap():
    rng = np.random.default_rng(4)
    P = rng.uniform(0, 255, (60, 3))
    c = P[seeding.distinct_indices(60, 7, 4)] + rng.normal(0, 3, (7, 3))
    sr = 50.0
    Kh = nystrom.nystrom_kernel_matrix(P, c, sr)
    # K_hat = B^T A^+ B with a library pseudo-inverse
    A = np.exp(-((c[:, None] - c[None]) ** 2).sum(-1) / (2 * sr * sr))
    Bm = np.exp(-((c[:, None] - P[None]) ** 2).sum(-1) / (2 * sr * sr))
    np.testing.assert_allclose(Kh, Bm.T @ np.linalg.pinv(A, rcond=1e-10) @ Bm, rtol=0, atol=1e-9)
    K = nystrom.kernel_matrix(P, sr)
    ev = np.linalg.eigvalsh(K - Kh)
    assert ev.min() > -1e-9                          # Schur complement is PSD
    assert np.diag(Kh).max() <= 1 + 1e-9
    assert np.linalg.matrix_rank(Kh, tol=1e-8) <= 7  # rank K_hat <= m0


def test_sum_switch_matches_pointwise_form():
    f = synth.rectangles_image(26, 22, 6, 20.0, seed=9).astype(np.float64)
    P = f.reshape(-1, 3)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], 10, 9)], 5)
    gh, eta = nystrom.nystrom_filter(f, f, c, 2.0, 30.0, 4, return_eta=True)
    coords = np.array([[0, 0], [25, 21], [12, 10], [3, 20], [20, 2]])
    gp, ep = nystrom.nystrom_filter_at(f, f, c, 2.0, 30.0, 4, coords)
    np.testing.assert_allclose(gp, gh[coords[:, 0], coords[:, 1]], rtol=0, atol=1e-9)
    np.testing.assert_allclose(ep, eta[coords[:, 0], coords[:, 1]], rtol=1e-11, atol=1e-12)


def test_box_kernel_and_patch_guide_pointwise():
    f = synth.rectangles_image(18, 20, 5, 25.0, seed=10).astype(np.float64)
    p = exact.patch_guide(f, 1)
    P = p.reshape(-1, p.shape[2])
    c = P[seeding.distinct_indices(P.shape[0], 12, 10)]
    gh = nystrom.nystrom_filter(f, p, c, 1.0, 80.0, 3, spatial="box")
    coords = np.array([[0, 0], [17, 19], [9, 9]])
    gp, _ = nystrom.nystrom_filter_at(f, p, c, 1.0, 80.0, 3, coords, spatial="box")
    np.testing.assert_allclose(gp, gh[coords[:, 0], coords[:, 1]], rtol=0, atol=1e-9)


def test_theorem_bound_holds():
    # Theorem (Section III) with the proof in the supplement: per pixel,
    # |g_hat - g| <= |W_x| * max|K_hat - K| * (|g_hat(x)| + R sqrt(n)) / k(0, 0),
    # using eta >= w(0) k(0,0) and |Delta(x, y)| <= max |K_hat - K|.
    f = synth.rectangles_image(20, 18, 6, 20.0, seed=11).astype(np.float64)
    P = f.reshape(-1, 3)
    S, ss, sr = 3, 1.5, 40.0
    for r in (3, 6, 12):
        c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, r)], 8)
        g = exact.exact_filter(f, f, ss, sr, S)
        gh = nystrom.nystrom_filter(f, f, c, ss, sr, S)
        dmax = np.abs(nystrom.nystrom_kernel_matrix(P, c, sr) - nystrom.kernel_matrix(P, sr)).max()
        err = np.linalg.norm(gh - g, axis=2)
        bound = (2 * S + 1) ** 2 * dmax * (np.linalg.norm(gh, axis=2) + 255.0 * np.sqrt(3.0))
        assert np.all(err <= bound)


def test_affine_and_transpose_equivariance():
    f = synth.rectangles_image(21, 19, 6, 20.0, seed=12).astype(np.float64)
    P = f.reshape(-1, 3)
    c = P[seeding.distinct_indices(P.shape[0], 8, 12)]
    gh = nystrom.nystrom_filter(f, f, c, 2.0, 35.0, 4)
    # the guide is held fixed; f is transformed
    ga = nystrom.nystrom_filter(2.5 * f + 7.0, f, c, 2.0, 35.0, 4)
    np.testing.assert_allclose(ga, 2.5 * gh + 7.0, rtol=1e-11, atol=1e-9)
    ft = f.transpose(1, 0, 2)
    gt = nystrom.nystrom_filter(ft, ft, c, 2.0, 35.0, 4)
    np.testing.assert_allclose(gt, gh.transpose(1, 0, 2), rtol=1e-11, atol=1e-9)


def test_accuracy_improves_with_landmarks_soft():
    # Supplement, PSNR vs m0: accuracy grows with the number of clusters.
    f, prm = synth.workload("color_blf_256", 64, 64)
    f = f.astype(np.float64)
    P = f.reshape(-1, 3)
    g = exact.exact_filter(f, f, prm["sigma_s"], prm["sigma_r"], prm["S"])
    ps = []
    for r in (2, 16):
        c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, 1)], 10)
        ps.append(exact.psnr(nystrom.nystrom_filter(f, f, c, prm["sigma_s"], prm["sigma_r"],
                                                    prm["S"]), g))
    assert ps[1] > ps[0] + 3.0
    assert ps[1] > 20.0


def test_guard_nonpositive_eta_outputs_input():
    # eta_hat can be <= 0 for a Nystrom kernel; such pixels output f (reading of
    # the normalisation step of Algorithm 1).  Force it with a negative-eigen-
    # direction guide: one landmark far from every pixel and tau = 0.
    f = np.arange(2 * 3 * 1, dtype=np.float64).reshape(2, 3, 1) + 1.0
    p = np.zeros((2, 3, 1))
    c = np.array([[1e6]])
    g, eta = nystrom.nystrom_filter(f, p, c, 1.0, 1.0, 1, tau=0.0, return_eta=True)
    assert np.all(eta == 0)
    np.testing.assert_array_equal(g, f)


def _perturbed_pipeline(f, p, c, sigma_s, sigma_r, S, spatial, delta, rng, perturb_b):
    """Algorithm 1 in FP64 with centring f~ = f - f0, every stored
    intermediate (u_k(x), u_k f~_c, the convolved planes, and b_j(x) when
    ``perturb_b``) multiplied by an independent random factor
    1 + delta * U(-1, 1)."""
    H, W, C = f.shape
    f0 = 0.5 * (f.min(axis=(0, 1)) + f.max(axis=(0, 1)))
    fc = f - f0
    w1 = exact.spatial_taps(sigma_s, S, spatial)
    alpha, Wv = nystrom.landmark_eig(c, sigma_r)
    Fm = Wv / np.sqrt(alpha)[None, :]

    def pert(a):
        return a * (1.0 + delta * rng.uniform(-1.0, 1.0, a.shape))

    b = nystrom.cross_kernel_sr(c, p.reshape(H * W, -1), sigma_r)
    if perturb_b:
        b = pert(b)
    U = pert(b @ Fm)
    zeta = np.zeros((H, W, C))
    eta = np.zeros((H, W))
    for k in range(U.shape[1]):
        uk = U[:, k].reshape(H, W)
        zeta += uk[:, :, None] * pert(nystrom.conv_zero(pert(uk[:, :, None] * fc), w1))
        eta += uk * pert(nystrom.conv_zero(uk, w1))
    return zeta / eta[:, :, None] + f0


@pytest.mark.parametrize("C,r,seed", [(3, 12, 1), (1, 12, 2), (1, 6, 3)])
@pytest.mark.parametrize("perturb_b", [False, True])
def test_storage_bound_covers_injected_perturbations(C, r, seed, perturb_b):
    """The per-pixel storage bound B (first order) covers the change of g_hat
    when each stored stage is perturbed by up to delta relative:
    |dg| <= 4 delta B (5 delta B with b).  The 1-D guide with 12 landmarks is
    ill-conditioned (Eq. (vk) cancels, |F| ~ 1e4): there a rounding of b is
    amplified far beyond |u_k|, which only the cross-kernel form of B covers
    (checked as well: the plain form is exceeded)."""
    rng = np.random.default_rng(seed)
    f, _ = synth.workload("color_blf_256", 24, 28, seed=600 + seed)
    f = np.ascontiguousarray(f[:, :, :C]).astype(np.float64)
    P = f.reshape(-1, C)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, seed)], 5)
    B = nystrom.storage_error_bound(f, f, c, 1.5, 30.0, 3, cross_kernel_rounding=perturb_b)
    g0 = _perturbed_pipeline(f, f, c, 1.5, 30.0, 3, "gaussian", 0.0, rng, perturb_b)
    delta, stages = 1e-9, (5 if perturb_b else 4)
    worst = 0.0
    for _ in range(3):
        g1 = _perturbed_pipeline(f, f, c, 1.5, 30.0, 3, "gaussian", delta, rng, perturb_b)
        ok = np.isfinite(B)
        worst = max(worst, float((np.abs(g1 - g0)[ok] / (stages * delta * B[ok])).max()))
    assert worst <= 1.0, worst
    if perturb_b and (C, r) == (1, 12):
        Bp = nystrom.storage_error_bound(f, f, c, 1.5, 30.0, 3)
        g1 = _perturbed_pipeline(f, f, c, 1.5, 30.0, 3, "gaussian", delta, rng, True)
        ok = np.isfinite(Bp)
        assert (np.abs(g1 - g0)[ok] / (stages * delta * Bp[ok])).max() > 1.0


@pytest.mark.parametrize("spatial", ["gaussian", "box"])
def test_storage_bound_at_pixels_equals_full_bound(spatial):
    """The window-by-window evaluation of the storage bound agrees with the
    whole-image one (which the perturbation test above pins) at interior,
    border and corner pixels."""
    f, _ = synth.workload("color_blf_256", 26, 31, seed=77)
    f = f.astype(np.float64)
    P = f.reshape(-1, 3)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], 9, 5)], 4)
    B = nystrom.storage_error_bound(f, f, c, 1.5, 30.0, 3, spatial)
    coords = np.array([[0, 0], [25, 30], [0, 30], [13, 17], [2, 3], [24, 1]])
    Bat = nystrom.storage_error_bound_at(f, f, c, 1.5, 30.0, 3, coords, spatial)
    np.testing.assert_allclose(Bat, B[coords[:, 0], coords[:, 1]], rtol=1e-9)
