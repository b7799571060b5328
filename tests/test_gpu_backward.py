"""GPU backward (hand-written adjoint) against the float64 autograd reference
of the same approximation (itself pinned to central finite differences and
to exact identities in test_oracle_grad.py).

Bar: every gradient entry within 2e-4 of the largest reference magnitude of
that gradient (relative max-norm).  The forward runs in FP32 with
FP64-accumulated convolutions; the adjoint is the same arithmetic, so its
error is of the same order as the forward's (~1e-7 relative per stored
value, amplified by the eta conditioning).  A sigma gradient is a sum over
all pixels of G * dg/dsigma whose terms cancel (by a factor of thousands for
sigma_s), so its bar is max(2e-4 |ref|, 4 * 2^-24 * sum |G dg/dsigma|): a few
FP32 roundings per term, with the scale taken from FP64 central differences
of the oracle forward.
"""
import numpy as np
import pytest
import torch

from oracle import grad, kmeans, nystrom, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu

RTOL_MAX = 2e-4


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _case(h, w, r, seed, iters=6):
    f, _ = synth.workload("diff_batch8", h, w, seed=seed)
    P = f.reshape(-1, 3).astype(np.float64)
    c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], r, seed)], iters)
    G = np.random.default_rng(seed).normal(0, 1, f.shape).astype(np.float32)
    return f, c.astype(np.float32), G


def _gpu_grads(f, p, c32, G, ss, sr, S, **kw):
    nkf = _nkf()
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), sr)
    ft = torch.from_numpy(f).cuda()
    pt = torch.from_numpy(np.ascontiguousarray(p)).cuda() if p is not None else None
    df, dp, dsr, dss = nkf.filter_backward(ft, torch.from_numpy(c32).cuda(), Q, al, reff,
                                           torch.from_numpy(G).cuda(), pt, sigma_s=ss, sigma_r=sr,
                                           radius=S, **kw)
    torch.cuda.synchronize()
    return df.cpu().numpy().astype(np.float64), dp.cpu().numpy().astype(np.float64), dsr, dss


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _sigma_scales(f, p, c32, G, ss, sr, S):
    """sum_x |G dg/dsigma| for sigma_r and sigma_s (FP64 oracle, central
    differences with step 1e-4 sigma)."""
    f64, p64, c64 = f.astype(np.float64), p.astype(np.float64), c32.astype(np.float64)

    def g(s_s, s_r):
        return nystrom.nystrom_filter(f64, p64, c64, s_s, s_r, S)
    hr, hs = 1e-4 * sr, 1e-4 * ss
    dr = (g(ss, sr + hr) - g(ss, sr - hr)) / (2 * hr)
    ds = (g(ss + hs, sr) - g(ss - hs, sr)) / (2 * hs)
    return np.abs(G * dr).sum(), np.abs(G * ds).sum()


def _sigma_ok(val, ref, scale):
    return abs(val - ref) <= max(RTOL_MAX * abs(ref), 4 * 2.0 ** -24 * scale)


# r = 48 and 64 take the reduction's 16-landmark register blocks (r > 32)
@pytest.mark.parametrize("h,w,r,S,ss,sr", [(40, 36, 12, 4, 1.5, 30.0), (75, 66, 32, 9, 3.0, 30.0),
                                           (44, 50, 8, 12, 4.0, 30.0), (38, 41, 6, 16, 5.0, 40.0),
                                           (64, 56, 48, 6, 2.0, 20.0), (72, 60, 64, 5, 2.0, 20.0)])
def test_explicit_guide_grads_match_reference(h, w, r, S, ss, sr):
    f, c32, G = _case(h, w, r, seed=h)
    p = np.ascontiguousarray(f + 0.0)
    df, dp, dsr, dss = _gpu_grads(f, p, c32, G, ss, sr, S)
    ref = grad.reference_grads(f.astype(np.float64), p.astype(np.float64), c32.astype(np.float64), ss, sr, S, G)
    e = dict(f=_rel(df, ref["f"]), p=_rel(dp, ref["p"]),
             sr=abs(dsr - ref["sigma_r"]) / abs(ref["sigma_r"]), ss=abs(dss - ref["sigma_s"]) / abs(ref["sigma_s"]))
    scr, scs = _sigma_scales(f, p, c32, G.astype(np.float64), ss, sr, S)
    print(f"[bwd {h}x{w} r{r} S{S}] rel errors {e}  (sigma_r {dsr:.6g} vs {ref['sigma_r']:.6g}, "
          f"sigma_s {dss:.6g} vs {ref['sigma_s']:.6g}; abs errors / sum|terms|: "
          f"{abs(dsr - ref['sigma_r']) / scr:.2e}, {abs(dss - ref['sigma_s']) / scs:.2e})", flush=True)
    assert e["f"] <= RTOL_MAX and e["p"] <= RTOL_MAX
    assert _sigma_ok(dsr, ref["sigma_r"], scr) and _sigma_ok(dss, ref["sigma_s"], scs)


def test_autograd_function_self_guided():
    nkf = _nkf()
    f, c32, G = _case(48, 40, 10, seed=7)
    ss, sr, S = 2.0, 35.0, 5
    ft = torch.from_numpy(f).cuda().requires_grad_(True)
    srt = torch.tensor(sr, dtype=torch.float64, requires_grad=True)
    sst = torch.tensor(ss, dtype=torch.float64, requires_grad=True)
    out = nkf.NystromFilter.apply(ft, None, srt, sst, torch.from_numpy(c32).cuda(), S)
    (out * torch.from_numpy(G).cuda()).sum().backward()
    ref = grad.reference_grads(f.astype(np.float64), f.astype(np.float64), c32.astype(np.float64), ss, sr, S, G)
    tot = ref["f"] + ref["p"]
    e = _rel(ft.grad.cpu().numpy().astype(np.float64), tot)
    print(f"[autograd self] rel df {e:.2e} sigma_r {float(srt.grad):.6g} vs {ref['sigma_r']:.6g}", flush=True)
    assert e <= RTOL_MAX
    scr, scs = _sigma_scales(f, f, c32, G.astype(np.float64), ss, sr, S)
    assert _sigma_ok(float(srt.grad), ref["sigma_r"], scr)
    assert _sigma_ok(float(sst.grad), ref["sigma_s"], scs)


def test_full_size_batch_image_invariants():
    """One image of the differentiation batch at its full drawn size:
    shift equivariance gives sum_x dL/df_c = sum_x G_c; finite outputs."""
    sizes = synth.batch_sizes()
    h, w = sizes[0]
    f, c32, G = _case(h, w, 32, seed=1050, iters=3)
    df, dp, dsr, dss = _gpu_grads(f, np.ascontiguousarray(f + 0.0), c32, G, 3.0, 30.0, 9)
    lhs = df.sum(axis=(0, 1))
    rhs = G.astype(np.float64).sum(axis=(0, 1))
    scale = np.abs(G).astype(np.float64).sum(axis=(0, 1))
    print(f"[bwd full {h}x{w}] sum df {lhs} vs sum G {rhs}", flush=True)
    assert np.all(np.abs(lhs - rhs) <= 1e-4 * scale)
    assert np.isfinite(df).all() and np.isfinite(dp).all() and np.isfinite(dsr) and np.isfinite(dss)


def test_constant_image_zero_guide_and_sigma_grads():
    nkf = _nkf()
    rng = np.random.default_rng(3)
    f = np.full((30, 34, 3), 90.0, np.float32)
    p = rng.uniform(0, 255, (30, 34, 3)).astype(np.float32)
    c32 = p.reshape(-1, 3)[seeding.distinct_indices(30 * 34, 6, 3)]
    G = rng.normal(0, 1, f.shape).astype(np.float32)
    df, dp, dsr, dss = _gpu_grads(f, p, c32, G, 1.5, 60.0, 3)
    assert np.abs(dp).max() <= 1e-6 * np.abs(df).max() + 1e-9
    assert abs(dsr) <= 1e-4 and abs(dss) <= 1e-4


def test_unsupported_backward_requests():
    nkf = _nkf()
    f = torch.rand(20, 20, 4, device="cuda") * 255
    c = f.reshape(-1, 4)[:5].contiguous()
    Q, al, F, reff = nkf.landmark_factor(c.cpu().numpy().astype(np.float64), 30.0)
    with pytest.raises(nkf.NkfError) as ei:
        nkf.filter_backward(f, c, Q, al, reff, torch.ones_like(f), sigma_s=2.0, sigma_r=30.0, radius=3)
    assert ei.value.status == nkf.NKF_ERR_UNSUPPORTED


def test_forward_outputs_reused_bitwise():
    """The backward fed the forward's own output and eta_hat (no convolution
    recompute) gives bit-identical gradients to the recomputing backward."""
    nkf = _nkf()
    f, c32, G = _case(57, 49, 16, seed=21)
    ss, sr, S = 2.0, 30.0, 6
    Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), sr)
    ft = torch.from_numpy(f).cuda()
    ct_ = torch.from_numpy(c32).cuda()
    Gt = torch.from_numpy(G).cuda()
    out, eta = nkf.filter_landmarks(ft, ct_, F, sigma_s=ss, sigma_r=sr, radius=S, return_eta=True)
    a = nkf.filter_backward(ft, ct_, Q, al, reff, Gt, sigma_s=ss, sigma_r=sr, radius=S)
    b = nkf.filter_backward(ft, ct_, Q, al, reff, Gt, sigma_s=ss, sigma_r=sr, radius=S, out=out, eta=eta)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert a[2] == b[2] and a[3] == b[3]
