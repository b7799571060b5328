"""GPU k-means (Section III landmarks) against the FP64 oracle.

k-means labels are not unique at near-ties, so parity is checked on what is
unique: the seeding gather is bit-exact; one Lloyd step from the same
centroids gives the oracle's labels wherever the two best squared distances
are not a float32 near-tie; the updated centroids equal the FP64 mean of the
members under the GPU's own labels, within the error of float32 partial sums
of at most 64 values (6 * 2^-24 relative, bound taken as 1e-6).
"""
import numpy as np
import pytest
import torch

from oracle import exact, kmeans, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _case(kind, h, w):
    if kind == "self3":
        f, prm = synth.workload("color_blf_2048", h, w)
        return f, None, "self", f.reshape(-1, 3).astype(np.float64)
    if kind == "explicit2":
        f, _ = synth.workload("color_blf_256", h, w)
        p = np.ascontiguousarray(f[:, :, :2])
        return f, p, "explicit", p.reshape(-1, 2).astype(np.float64)
    if kind == "hyper":
        f, _ = synth.workload("hyperspectral_512x128", h, w)
        return f, None, "self", f.reshape(-1, f.shape[2]).astype(np.float64)
    if kind == "explicit25":
        f, _ = synth.workload("color_blf_256", h, w)
        p = np.ascontiguousarray(synth.workload("hyperspectral_512x128", h, w)[0][:, :, :25] * 255.0)
        return f, p, "explicit", p.reshape(-1, 25).astype(np.float64)
    if kind in ("patch", "patch2"):
        f, _ = synth.workload("color_nlm_1024", h, w)
        pg = exact.patch_guide(f.astype(np.float64), 3 if kind == "patch" else 2)
        return f, None, "patch", pg.reshape(-1, pg.shape[2])
    raise KeyError(kind)


def _near_tie(P, c, rel=2e-5):
    d2 = np.stack([((P - ck) ** 2).sum(1) for ck in c], 1)
    s = np.sort(d2, 1)
    scale = (P * P).sum(1) + (c * c).sum(1).max()
    return (s[:, 1] - s[:, 0]) <= rel * scale + 1e-6


# explicit25: D + 1 <= 64 (several pixels per wave instruction in the FP32 sums);
# hyper and patch: D + 1 > 64 (64-dimension slices); hyper with r = 256: the
# FP32 sums do not fit in LDS (FP64 sums in the block's slot); patch2 (5x5x3
# patches, D + 1 = 76): three pixel stripes per block in the sums, each
# crossing image rows of an odd width.  The FP32 labels of D > 32 come from the
# matrix cores: 4, 8 and 16 landmark tiles (r = 64, 128, 256 with patch2); hyper
# with r = 256 does not fit their LDS tile and takes the VALU kernel
@pytest.mark.parametrize("kind,h,w,r", [("self3", 70, 90, 32), ("explicit2", 64, 64, 8),
                                         ("explicit25", 50, 46, 31), ("hyper", 40, 36, 64),
                                         ("hyper", 40, 36, 256), ("patch", 48, 40, 128),
                                         ("patch2", 37, 53, 16), ("patch2", 41, 47, 256)])
def test_seed_and_one_lloyd_step(kind, h, w, r):
    nkf = _nkf()
    f, p, guide, P = _case(kind, h, w)
    ft = torch.from_numpy(f).cuda()
    pt = torch.from_numpy(p).cuda() if p is not None else None
    pk = {"patch_radius": 2} if kind == "patch2" else {}
    c0 = nkf.kmeans(ft, pt, r=r, iters=0, seed=11, guide=guide, **pk)
    torch.cuda.synchronize()
    idx = seeding.distinct_indices(P.shape[0], r, 11)
    np.testing.assert_array_equal(c0.cpu().numpy(), P[idx].astype(np.float32))
    c_start = c0.cpu().numpy().astype(np.float64)
    c1, lab = nkf.kmeans_iterate(ft, c0, pt, iters=1, guide=guide, return_labels=True, **pk)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy().reshape(-1)
    lab_or, _ = kmeans.assign(P, c_start)
    tie = _near_tie(P, c_start)
    mism = (lab != lab_or) & ~tie
    print(f"[{kind}] label mismatches outside near-ties: {mism.sum()} (near-ties {tie.sum()})", flush=True)
    assert mism.sum() == 0
    c_or, _, cnt = kmeans.update(P, lab.astype(np.int64), c_start)
    c1 = c1.cpu().numpy().astype(np.float64)
    scale = np.abs(P).max()
    np.testing.assert_allclose(c1, c_or.astype(np.float32).astype(np.float64), rtol=0, atol=1e-6 * scale)


def test_objective_non_increasing_on_gpu():
    nkf = _nkf()
    f, _ = synth.workload("color_blf_256", 96, 96)
    P = f.reshape(-1, 3).astype(np.float64)
    ft = torch.from_numpy(f).cuda()
    c = nkf.kmeans(ft, r=16, iters=0, seed=1)
    errs = []
    for _ in range(8):
        errs.append(kmeans.quantization_error(P, c.cpu().numpy().astype(np.float64)))
        nkf.kmeans_iterate(ft, c, iters=1)
    errs.append(kmeans.quantization_error(P, c.cpu().numpy().astype(np.float64)))
    assert all(b <= a * (1 + 1e-6) for a, b in zip(errs, errs[1:])), errs


def test_full_size_color_2048_one_step():
    nkf = _nkf()
    f, prm = synth.workload("color_blf_2048")
    P = f.reshape(-1, 3).astype(np.float64)
    ft = torch.from_numpy(f).cuda()
    c0 = nkf.kmeans(ft, r=32, iters=0, seed=prm["landmark_seed"])
    c_start = c0.cpu().numpy().astype(np.float64)
    c1, lab = nkf.kmeans_iterate(ft, c0, iters=1, return_labels=True)
    lab = lab.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(5)
    samp = rng.integers(0, P.shape[0], 20000)
    lab_or, _ = kmeans.assign(P[samp], c_start)
    tie = _near_tie(P[samp], c_start)
    assert ((lab[samp] != lab_or) & ~tie).sum() == 0
    c_or, _, _ = kmeans.update(P, lab.astype(np.int64), c_start)
    np.testing.assert_allclose(c1.cpu().numpy().astype(np.float64), c_or.astype(np.float32).astype(np.float64),
                               rtol=0, atol=1e-6 * 255)
