"""The allocation-free forward entry point against the allocating one.

nkf_filter_landmarks_noalloc runs the kernels of nkf_filter_landmarks with
its scratch in the library's fixed device array instead of the context's
workspace.  Both are called through the C ABI on the same inputs, several
calls in a row with shrinking inputs (the array keeps the previous call's
contents), and must agree within the FP32 path's 1e-4 bar (0-255 scale).
"""
import ctypes as ct

import numpy as np
import pytest
import torch

from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _landmarks(nkf, f, r, guide, patch_radius, sigma_r, precision="fp32"):
    c = nkf.kmeans(f, r=r, iters=3, seed=5, guide=guide, patch_radius=patch_radius, precision=precision)
    _, _, F, r_eff = nkf.landmark_factor(c, sigma_r)
    return c, torch.from_numpy(F).to(f.device), r_eff


def _both(nkf, f, c, F, r_eff, prm, D):
    """(out, eta) of the allocating and of the allocation-free entry point."""
    lib = nkf.load_library()
    ctx = nkf._cur_ctx(f)
    H, W, C = f.shape
    res = []
    for fn in (lib.nkf_filter_landmarks, lib.nkf_filter_landmarks_noalloc):
        out = torch.full_like(f, -9.0)
        eta = torch.full((H, W), -9.0, dtype=torch.float32, device=f.device)
        st = fn(ctx, H, W, C, ct.c_void_p(f.data_ptr()), D, ct.c_void_p(0), ct.byref(prm),
                ct.c_void_p(c.data_ptr()), ct.c_void_p(F.data_ptr()), int(r_eff), ct.c_void_p(out.data_ptr()),
                ct.c_void_p(eta.data_ptr()))
        assert st == nkf.NKF_OK, lib.nkf_last_error(ctx)
        res.append((out, eta))
    torch.cuda.synchronize()
    return res


CASES = [
    # (H, W, r, spatial, guide, patch_radius, precision, sigma_s, sigma_r, radius)
    (160, 136, 24, "gaussian", "self", 0, "fp32", 3.0, 30.0, 9),
    (72, 58, 12, "gaussian", "self", 0, "fp32", 2.0, 25.0, 6),
    (96, 70, 32, "box", "patch", 1, "fp16", 1.0, 60.0, 4),
    (37, 45, 8, "box", "patch", 1, "fp32", 1.0, 60.0, 3),
]


def test_noalloc_matches_allocating_entry_point():
    nkf = _nkf()
    dev = torch.device("cuda:0")
    for i, (H, W, r, spatial, guide, pr, prec, ss, sr, rad) in enumerate(CASES):
        print(f"case {i}: {H}x{W} r={r} {spatial} {guide} {prec}", flush=True)
        f = torch.from_numpy(synth.rectangles_image(H, W, 3, 20.0, seed=40 + i)).to(dev)
        D = 3 if guide == "self" else 3 * (2 * pr + 1) ** 2
        c, F, r_eff = _landmarks(nkf, f, r, guide, pr, sr, prec)
        prm = nkf.make_params(sigma_s=ss, sigma_r=sr, r=r, radius=rad, spatial=spatial, guide=guide,
                              patch_radius=pr, precision=prec)
        (o1, e1), (o2, e2) = _both(nkf, f, c, F, r_eff, prm, D)
        assert torch.isfinite(o1).all()
        d_out = float((o1 - o2).abs().max())
        d_eta = float((e1 - e2).abs().max())
        print(f"  max |out diff| = {d_out:.3e}, max |eta diff| = {d_eta:.3e}", flush=True)
        assert d_out <= TOL and d_eta <= TOL * 1e-2


def test_noalloc_rejects_problems_beyond_its_scratch():
    nkf = _nkf()
    lib = nkf.load_library()
    dev = torch.device("cuda:0")
    # 1024 x 1024 pixels with 32 embedding planes need 128 MiB of scratch
    H = W = 1024
    f = torch.zeros((H, W, 3), dtype=torch.float32, device=dev)
    c = torch.zeros((32, 3), dtype=torch.float32, device=dev)
    F = torch.eye(32, dtype=torch.float64, device=dev)
    out = torch.full_like(f, -5.0)
    prm = nkf.make_params(sigma_s=3.0, sigma_r=30.0, r=32, radius=9)
    ctx = nkf._cur_ctx(f)
    st = lib.nkf_filter_landmarks_noalloc(ctx, H, W, 3, ct.c_void_p(f.data_ptr()), 3, ct.c_void_p(0),
                                          ct.byref(prm), ct.c_void_p(c.data_ptr()), ct.c_void_p(F.data_ptr()), 32,
                                          ct.c_void_p(out.data_ptr()), ct.c_void_p(0))
    assert st == nkf.NKF_ERR_OUT_OF_MEMORY
    assert b"static scratch" in lib.nkf_last_error(ctx)
    torch.cuda.synchronize()
    assert bool((out == -5.0).all())
