"""Oracle parity of the convolution kernels at the tile geometry of the large
workloads (Algorithm 1, Section III).

Each block of the Gaussian-window kernels (forward and backward) streams its
output tile in chunks of rows through an LDS ring; small images get one
chunk per tile, large ones up to eight, so the ring wraps only there.  These
tests force the chunk counts of the large workloads (nkf_set_conv_chunks) on
images the oracle handles in full, and compare sampled pixels of the
full-size workloads, in their own launch configuration, with the oracle
evaluated pixel by pixel.  The box-window kernel has fixed tiles of 56 (or
48) rows and is checked here on images with partial tiles in both
directions.

Bars as in test_gpu_parity.py: 1e-4 on the 0-255 scale (1e-4 / 255 on the
[0, 1] hyperspectral scale) on every pixel whose first-order FP32 storage
bound is below it and the rest within that bound; the box window (FP64
throughout) 1e-4 on every pixel.
"""
import contextlib

import numpy as np
import pytest
import torch

from oracle import exact, grad, kmeans, nystrom, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu

TOL_255 = 1e-4
EPS_STORE = 4 * 2.0 ** -24


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


@contextlib.contextmanager
def _chunks(t, n):
    nkf = _nkf()
    nkf.set_conv_chunks(t, n)
    try:
        yield
    finally:
        nkf.set_conv_chunks(t, 0)


def _landmarks(P, r, seed, iters):
    c0 = P[seeding.distinct_indices(P.shape[0], r, seed)]
    c, _, _ = kmeans.lloyd(P, c0, iters)
    return c.astype(np.float32)


def _sample_landmarks(P, r, seed, iters, n=16384):
    """Oracle k-means on n pixels drawn by the seeding draw (large images)."""
    return _landmarks(P[seeding.distinct_indices(P.shape[0], n, seed + 100)], r, seed, iters)


def _grade(name, g, go, bound, tol):
    """g, go, bound: [..., C].  1e-4-type bar where the bound allows it."""
    err = np.abs(g - go)
    well = EPS_STORE * bound <= tol
    n_ill = int((~well).sum())
    i = np.unravel_index(np.argmax(err), err.shape)
    print(f"[{name}] max|dg|={err.max():.3e} at {i}; well-conditioned ({int(well.sum())}) max|dg|="
          f"{err[well].max() if well.any() else 0.0:.3e}; ill-conditioned entries {n_ill}"
          + (f", max|dg|/bound={np.max(err[~well] / (EPS_STORE * bound[~well])):.3f}" if n_ill else ""),
          flush=True)
    if well.any():
        assert err[well].max() <= tol, name
    if n_ill:
        assert np.all(err[~well] <= EPS_STORE * bound[~well]), name


def _grade_box(name, g, go, tol):
    """Box window: FP64 from the embedding planes to the output, so 1e-4 on
    every entry."""
    err = np.abs(g - go)
    i = np.unravel_index(np.argmax(err), err.shape)
    print(f"[{name}] max|dg|={err.max():.3e} at {i} over {err.size} entries", flush=True)
    assert err.max() <= tol, name


def _filter(f, p, c32, sigma_s, sigma_r, S, nch, **kw):
    nkf = _nkf()
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), sigma_r)
    ft = torch.from_numpy(np.ascontiguousarray(f, np.float32)).cuda()
    pt = torch.from_numpy(np.ascontiguousarray(p, np.float32)).cuda() if p is not None else None
    ct_ = torch.from_numpy(c32).cuda()
    with _chunks(ft, nch):
        g = nkf.filter_landmarks(ft, ct_, F, pt, sigma_s=sigma_s, sigma_r=sigma_r, radius=S, **kw)
    g_auto = nkf.filter_landmarks(ft, ct_, F, pt, sigma_s=sigma_s, sigma_r=sigma_r, radius=S, **kw)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    print(f"  forced {nch} chunks vs automatic: max|dg|={np.abs(g - g_auto.cpu().numpy()).max():.3e}", flush=True)
    return g


def test_box_patch_guide_tiles():
    """The colour NLM kernel (21 x 21 box, 7 x 7 x 3 patches): 300 x 72 pixels
    leave partial tiles in both directions; the FP32 form keeps the planes in
    FP64."""
    f, prm = synth.workload("color_nlm_1024", 300, 72)
    pg = exact.patch_guide(f.astype(np.float64), prm["patch_radius"])
    c32 = _landmarks(pg.reshape(-1, pg.shape[2]), 32, prm["landmark_seed"], 4)
    g = _filter(f, None, c32, 1.0, prm["sigma_r"], prm["S"], 0, spatial="box", guide="patch",
                patch_radius=prm["patch_radius"])
    go = nystrom.nystrom_filter(f.astype(np.float64), pg, c32.astype(np.float64), 1.0, prm["sigma_r"],
                                prm["S"], "box")
    _grade_box("box_patch", g, go, TOL_255)


@pytest.mark.parametrize("C", [3, 1])
def test_box_self_guide_tiles(C):
    f, _ = synth.workload("color_blf_256", 270, 45, seed=31)
    f = np.ascontiguousarray(f[:, :, :C])
    c32 = _landmarks(f.reshape(-1, C).astype(np.float64), 12, 3, 5)
    g = _filter(f, None, c32, 1.0, 30.0, 7, 0, spatial="box", guide="self")
    go = nystrom.nystrom_filter(f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64), 1.0,
                                30.0, 7, "box")
    _grade_box(f"box_C{C}", g, go, TOL_255)


@pytest.mark.parametrize("nch", [3, 8])
def test_gaussian_colour_multichunk(nch):
    """The headline kernel (Gaussian, E + 3 channel planes) at 8 chunks per
    tile, the 2048^2 workload's geometry."""
    f, prm = synth.workload("color_blf_2048", 2048, 2048)
    f = np.ascontiguousarray(f[500:780, 300:370])
    c32 = _landmarks(f.reshape(-1, 3).astype(np.float64), prm["r"], prm["landmark_seed"], 6)
    g = _filter(f, None, c32, prm["sigma_s"], prm["sigma_r"], prm["S"], nch, guide="self")
    go = nystrom.nystrom_filter(f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64),
                                prm["sigma_s"], prm["sigma_r"], prm["S"])
    B = nystrom.storage_error_bound(f, f, c32.astype(np.float64), prm["sigma_s"], prm["sigma_r"], prm["S"])
    _grade(f"gauss_C3_nch{nch}", g, go, B, TOL_255)


@pytest.mark.parametrize("nch", [2, 8])
def test_channel_chunks_multichunk(nch):
    """The C > 3 kernels (eta pass, then 4-channel chunks reading planar f,
    16-byte ring stores) of the hyperspectral workload at its 8 chunks per
    tile; 16 bands of the hyperspectral cube keep the oracle quick."""
    f, prm = synth.workload("hyperspectral_512x128", 270, 40)
    f = np.ascontiguousarray(f[:, :, ::8])
    c32 = _landmarks(f.reshape(-1, f.shape[2]).astype(np.float64), 24, prm["landmark_seed"], 4)
    g = _filter(f, f, c32, prm["sigma_s"], prm["sigma_r"], prm["S"], nch)
    go = nystrom.nystrom_filter(f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64),
                                prm["sigma_s"], prm["sigma_r"], prm["S"])
    B = nystrom.storage_error_bound(f, f, c32.astype(np.float64), prm["sigma_s"], prm["sigma_r"], prm["S"])
    _grade(f"chan16_nch{nch}", g, go, B, TOL_255 / 255)


@pytest.mark.parametrize("nch", [3, 8])
def test_backward_multichunk(nch):
    """Backward conv modes (du_dir, the fused sigma_s pass, the adjoint) with
    the ring wrapping, as on the 1016 x 574 and 959 x 883 batch images
    (r = 32 landmarks from 10 Lloyd iterations), against the float64
    autograd reference.  The reference has no eta <= 0 guard, so the case is
    one whose eta_hat stays well away from zero (checked with the oracle)."""
    nkf = _nkf()
    h, w, r, S, ss, sr, seed = 270, 40, 32, 9, 3.0, 30.0, 1050
    f, _ = synth.workload("diff_batch8", h, w, seed=seed)
    P = f.reshape(-1, 3).astype(np.float64)
    c32 = _landmarks(P, r, seed, 10)
    f64, c64 = f.astype(np.float64), c32.astype(np.float64)
    _, eta = nystrom.nystrom_filter(f64, f64, c64, ss, sr, S, return_eta=True)
    assert eta.min() > 1e-2 * eta.max()
    G = np.random.default_rng(5).normal(0, 1, f.shape).astype(np.float32)
    Q, al, F, reff = nkf.landmark_factor(c64, sr)
    ft = torch.from_numpy(f).cuda()
    pt = torch.from_numpy(np.ascontiguousarray(f + 0.0)).cuda()
    with _chunks(ft, nch):
        df, dp, dsr, dss = nkf.filter_backward(ft, torch.from_numpy(c32).cuda(), Q, al, reff,
                                               torch.from_numpy(G).cuda(), pt, sigma_s=ss, sigma_r=sr, radius=S)
    torch.cuda.synchronize()
    ref = grad.reference_grads(f64, f64, c64, ss, sr, S, G)

    def rel(a, b):
        return np.abs(a - b).max() / np.abs(b).max()
    ef = rel(df.cpu().numpy().astype(np.float64), ref["f"])
    ep = rel(dp.cpu().numpy().astype(np.float64), ref["p"])
    # sigma gradients sum terms that cancel: bar max(2e-4 |ref|, 4 * 2^-24 * sum |G dg/dsigma|),
    # the scale from FP64 central differences of the oracle forward
    hr, hs = 1e-4 * sr, 1e-4 * ss
    G64 = G.astype(np.float64)
    scr = np.abs(G64 * (nystrom.nystrom_filter(f64, f64, c64, ss, sr + hr, S)
                        - nystrom.nystrom_filter(f64, f64, c64, ss, sr - hr, S)) / (2 * hr)).sum()
    scs = np.abs(G64 * (nystrom.nystrom_filter(f64, f64, c64, ss + hs, sr, S)
                        - nystrom.nystrom_filter(f64, f64, c64, ss - hs, sr, S)) / (2 * hs)).sum()
    esr, ess = abs(dsr - ref["sigma_r"]), abs(dss - ref["sigma_s"])
    print(f"[bwd nch{nch}] rel df {ef:.2e} dp {ep:.2e}; |d sigma_r err| {esr:.3e} (ref {ref['sigma_r']:.6g}, "
          f"scale {scr:.3e}); |d sigma_s err| {ess:.3e} (ref {ref['sigma_s']:.6g}, scale {scs:.3e})", flush=True)
    assert ef <= 2e-4 and ep <= 2e-4
    assert esr <= max(2e-4 * abs(ref["sigma_r"]), EPS_STORE * scr)
    assert ess <= max(2e-4 * abs(ref["sigma_s"]), EPS_STORE * scs)


def _sampled_coords(H, W, n, seed):
    rng = np.random.default_rng(seed)
    # corners, Gaussian-kernel chunk and tile edges (32-row chunks, 32-column
    # tiles), box-kernel tile edges (48 or 56 rows, 44 columns at S = 10)
    edges = [[0, 0], [H - 1, W - 1], [0, W - 1], [H - 1, 0], [127, 31], [128, 32], [255, 33],
             [256, 64], [127, 500 % W], [128, 95], [383, 63], [384, 64], [511, 127], [512, 128],
             [47, 43], [48, 44], [55, 87], [56, 88], [95, 131], [96, 132], [111, 43], [112, 44]]
    edges = [[min(y, H - 1), min(x, W - 1)] for y, x in edges]
    return np.concatenate([rng.integers(0, [H, W], (n, 2)), np.array(edges)])


def test_full_size_nlm_1024_sampled():
    """The colour NLM workload at 1024^2 (21 x 21 box, 7 x 7 x 3 patches,
    r = 128) in the bench's launch configuration, including pixels on the
    tile and chunk boundaries, against the oracle pixel by pixel."""
    nkf = _nkf()
    f, prm = synth.workload("color_nlm_1024")
    ft = torch.from_numpy(f).cuda()
    kw = dict(guide="patch", patch_radius=prm["patch_radius"])
    pg = exact.patch_guide(f.astype(np.float64), prm["patch_radius"])
    c32 = _sample_landmarks(pg.reshape(-1, pg.shape[2]), prm["r"], prm["landmark_seed"], 3)
    c = torch.from_numpy(c32).cuda()
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), prm["sigma_r"])
    g = nkf.filter_landmarks(ft, c, F, sigma_s=1.0, sigma_r=prm["sigma_r"], radius=prm["S"], spatial="box", **kw)
    g = g.cpu().numpy().astype(np.float64)
    H, W = f.shape[:2]
    coords = _sampled_coords(H, W, 30, 1)
    args = (f.astype(np.float64), pg, c32.astype(np.float64), 1.0, prm["sigma_r"], prm["S"], coords)
    go, _ = nystrom.nystrom_filter_at(*args, spatial="box")
    _grade_box("nlm1024_sampled", g[coords[:, 0], coords[:, 1]], go, TOL_255)
    assert np.isfinite(g).all()


def test_full_size_hyperspectral_512_sampled():
    """The hyperspectral workload at 512^2 x 128 (r = 64, 25 x 25 Gaussian) in
    the bench's launch configuration (eta pass, then 32 channel chunks of 8
    row chunks per tile), against the oracle pixel by pixel."""
    nkf = _nkf()
    f, prm = synth.workload("hyperspectral_512x128")
    ft = torch.from_numpy(f).cuda()
    c32 = _sample_landmarks(f.reshape(-1, f.shape[2]).astype(np.float64), prm["r"], prm["landmark_seed"], 3)
    c = torch.from_numpy(c32).cuda()
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), prm["sigma_r"])
    g = nkf.filter_landmarks(ft, c, F, sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], radius=prm["S"])
    g = g.cpu().numpy().astype(np.float64)
    H, W = f.shape[:2]
    coords = _sampled_coords(H, W, 30, 2)
    args = (f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64), prm["sigma_s"], prm["sigma_r"],
            prm["S"], coords)
    go, _ = nystrom.nystrom_filter_at(*args)
    B = nystrom.storage_error_bound_at(*args)
    _grade("hyper512_sampled", g[coords[:, 0], coords[:, 1]], go, B, TOL_255 / 255)
    assert np.isfinite(g).all()
