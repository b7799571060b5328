"""GPU PCA patch guide (PCA-NLM, Section IV) against the FP64 oracle.

The device forms the sample moments in FP64, decomposes the covariance with
the library's host eigensolver and projects in FP64, storing float32.  Bars:
kept eigenvalues within 1e-10 relative; every guide entry of a component
whose eigenvalue is isolated (relative gap > 1e-6 to its neighbours) within
8 float32 roundings of the largest guide magnitude; and, for the whole kept
subspace (rotation within near-equal eigenvalues is not fixed by the
definition), squared distances between guide values within 1e-5 of the
largest one.
"""
import ctypes as ct

import numpy as np
import pytest
import torch

from oracle import exact, kmeans, nystrom, pca, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _check_guide(g_gpu, g_or, lam_or, label):
    H, W, dim = g_or.shape
    G, Go = g_gpu.reshape(-1, dim).astype(np.float64), g_or.reshape(-1, dim)
    scale = np.abs(Go).max()
    iso = []
    for k in range(dim):
        gaps = [abs(lam_or[k] - lam_or[j]) for j in (k - 1, k + 1) if 0 <= j < dim]
        if min(gaps) > 1e-6 * lam_or[0]:
            iso.append(k)
    err = np.abs(G[:, iso] - Go[:, iso]).max() if iso else 0.0
    rng = np.random.default_rng(0)
    sel = rng.choice(G.shape[0], size=min(300, G.shape[0]), replace=False)
    dG = ((G[sel, None, :] - G[None, sel, :]) ** 2).sum(-1)
    dO = ((Go[sel, None, :] - Go[None, sel, :]) ** 2).sum(-1)
    derr = np.abs(dG - dO).max() / dO.max()
    print(f"[pca {label}] isolated components {len(iso)}/{dim}: max err {err:.3e} (scale {scale:.3g}); "
          f"distance rel err {derr:.2e}", flush=True)
    assert err <= 8 * 2.0 ** -24 * scale
    assert derr <= 1e-5


@pytest.mark.parametrize("h,w,C,pr,dim", [(70, 66, 3, 3, 25), (45, 52, 3, 3, 6), (40, 37, 1, 2, 9)])
def test_guide_matches_oracle(h, w, C, pr, dim):
    nkf = _nkf()
    f, _ = synth.workload("color_nlm_1024", h, w, seed=h)
    f = np.ascontiguousarray(f[:, :, :C])
    g, ev = nkf.patch_pca(torch.from_numpy(f).cuda(), patch_radius=pr, dim=dim, seed=5, return_eigvals=True)
    torch.cuda.synchronize()
    g_or, lam = pca.pca_guide(f.astype(np.float64), pr, dim, seed=5)
    np.testing.assert_allclose(ev, lam, rtol=1e-10, atol=1e-12 * lam[0])
    _check_guide(g.cpu().numpy(), g_or, lam, f"{h}x{w}x{C} pr{pr} dim{dim}")


def test_large_image_uses_the_seeded_sample():
    """H*W > 65536: the basis comes from the SplitMix64 draw (same as the oracle)."""
    nkf = _nkf()
    f, _ = synth.workload("color_nlm_1024", 300, 262, seed=9)
    g, ev = nkf.patch_pca(torch.from_numpy(f).cuda(), patch_radius=1, dim=6, seed=77, return_eigvals=True)
    torch.cuda.synchronize()
    g_or, lam = pca.pca_guide(f.astype(np.float64), 1, 6, seed=77)
    np.testing.assert_allclose(ev, lam, rtol=1e-10, atol=1e-12 * lam[0])
    _check_guide(g.cpu().numpy(), g_or, lam, "300x262 sampled")


def test_pca_nlm_filter_matches_oracle():
    """The reduced guide drives the explicit-guide filter: FP32 path against
    the FP64 oracle evaluated with the same guide and landmarks."""
    nkf = _nkf()
    f, prm = synth.workload("color_nlm_1024", 48, 44, seed=3)
    ft = torch.from_numpy(f).cuda()
    g = nkf.patch_pca(ft, patch_radius=3, dim=25, seed=1)
    g64 = g.cpu().numpy().astype(np.float64)
    P = g64.reshape(-1, 25)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], 12, 2)], 5)
    c32 = c.astype(np.float32)
    sr = 400.0  # every pixel well conditioned: 4 eps B <= 7.4e-5 (storage bound)
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), sr)
    out = nkf.filter_landmarks(ft, torch.from_numpy(c32).cuda(), F, g, sigma_s=1.0, sigma_r=sr, radius=4,
                               spatial="box", guide="explicit")
    torch.cuda.synchronize()
    go = nystrom.nystrom_filter(f.astype(np.float64), g64, c32.astype(np.float64), 1.0, sr, 4, "box")
    err = np.abs(out.cpu().numpy().astype(np.float64) - go).max()
    print(f"[pca-nlm filter] max|dg| = {err:.3e}", flush=True)
    assert err <= 1e-4


def test_patch_pca_validation():
    nkf = _nkf()
    lib = nkf.load_library()
    f = torch.rand(20, 22, 3, device="cuda") * 255
    g = torch.empty(20 * 22 * 40, device="cuda")
    ctx = nkf._cur_ctx(f)

    def call(pr, dim):
        return lib.nkf_patch_pca(ctx, 20, 22, 3, ct.c_void_p(f.data_ptr()), pr, dim, 0, ct.c_void_p(g.data_ptr()),
                                 None)
    assert call(3, 33) == nkf.NKF_ERR_INVALID_ARG      # dim > 32
    assert call(1, 28) == nkf.NKF_ERR_INVALID_ARG      # dim > D = 27
    assert call(1, 0) == nkf.NKF_ERR_INVALID_ARG
    assert call(5, 10) == nkf.NKF_ERR_UNSUPPORTED      # D = 363 > 256
    assert call(-1, 4) == nkf.NKF_ERR_INVALID_ARG
    assert call(1, 27) == nkf.NKF_OK
