"""Python binding of the C ABI in include/nkf.h (ctypes, argument marshalling
only).  Every step of the filter runs in the HIP library; PyTorch provides
device memory and the current stream.  If the library is missing the calls
raise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnkf.so")

NKF_OK, NKF_ERR_INVALID_ARG, NKF_ERR_OUT_OF_MEMORY, NKF_ERR_HIP, NKF_ERR_NUMERICAL, NKF_ERR_UNSUPPORTED = range(6)
_STATUS = {1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "HIP", 4: "NUMERICAL", 5: "UNSUPPORTED"}

SPATIAL = {"gaussian": 0, "box": 1, "recursive": 2}
GUIDE = {"explicit": 0, "self": 1, "patch": 2}
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}

# every symbol the header declares
EXPORTS = [
    "nkf_params_default", "nkf_version", "nkf_create", "nkf_set_stream", "nkf_destroy",
    "nkf_last_error", "nkf_set_workspace_limit", "nkf_workspace_bytes", "nkf_filter", "nkf_kmeans",
    "nkf_kmeans_iterate", "nkf_landmark_factor", "nkf_filter_landmarks", "nkf_filter_backward",
    "nkf_seed_indices", "nkf_spatial_taps", "nkf_enable_timing", "nkf_stage_times", "nkf_patch_pca",
    "nkf_set_conv_chunks", "nkf_filter_landmarks_noalloc", "nkf_enable_stats", "nkf_get_stats",
]
STAGES = ["seed", "kmeans", "factor", "embed", "conv", "backward"]


class NkfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nkf error {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ct.Structure):
    _fields_ = [
        ("sigma_s", ct.c_double), ("sigma_r", ct.c_double), ("r", ct.c_int), ("radius", ct.c_int),
        ("spatial", ct.c_int), ("guide", ct.c_int), ("patch_radius", ct.c_int), ("prec", ct.c_int),
        ("kmeans_iters", ct.c_int), ("seed", ct.c_uint64), ("eig_rel_tol", ct.c_double),
        ("center", ct.c_double),
    ]


class Stats(ct.Structure):
    _fields_ = [
        ("valid", ct.c_int), ("r", ct.c_int), ("r_eff", ct.c_int), ("alpha_max", ct.c_double),
        ("alpha_min_kept", ct.c_double), ("cond_kept", ct.c_double), ("pixels", ct.c_longlong),
        ("guarded", ct.c_longlong), ("min_eta", ct.c_double),
    ]


_lib = None
_lib_lock = threading.Lock()


def load_library(path=LIB_PATH):
    """Load libnkf.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} (run python -m paper_1901_06112_amd.build)")
        lib = ct.CDLL(path)
        P, I, D, U64, SZ = ct.c_void_p, ct.c_int, ct.c_double, ct.c_uint64, ct.c_size_t
        PP = ct.POINTER(Params)
        sig = {
            "nkf_params_default": (None, [PP]),
            "nkf_version": (ct.c_char_p, []),
            "nkf_create": (I, [ct.POINTER(P), P]),
            "nkf_set_stream": (I, [P, P]),
            "nkf_destroy": (I, [P]),
            "nkf_last_error": (ct.c_char_p, [P]),
            "nkf_set_workspace_limit": (I, [P, SZ]),
            "nkf_workspace_bytes": (SZ, [P]),
            "nkf_filter": (I, [P, I, I, I, P, I, P, PP, P, P, ct.POINTER(I)]),
            "nkf_kmeans": (I, [P, I, I, I, P, I, P, PP, P, P]),
            "nkf_kmeans_iterate": (I, [P, I, I, I, P, I, P, PP, P, I, P]),
            "nkf_landmark_factor": (I, [I, I, P, D, D, P, P, P, ct.POINTER(I)]),
            "nkf_filter_landmarks": (I, [P, I, I, I, P, I, P, PP, P, P, I, P, P]),
            "nkf_filter_landmarks_noalloc": (I, [P, I, I, I, P, I, P, PP, P, P, I, P, P]),
            "nkf_filter_backward": (I, [P, I, I, I, P, I, P, PP, P, P, P, I, P, P, P, P, P, P, P]),
            "nkf_seed_indices": (I, [ct.c_int64, I, U64, P]),
            "nkf_spatial_taps": (I, [I, D, I, ct.POINTER(I), P]),
            "nkf_patch_pca": (I, [P, I, I, I, P, I, I, U64, P, P]),
            "nkf_enable_timing": (I, [P, I]),
            "nkf_stage_times": (I, [P, P, P, I]),
            "nkf_set_conv_chunks": (I, [P, I]),
            "nkf_enable_stats": (I, [P, I]),
            "nkf_get_stats": (I, [P, ct.POINTER(Stats)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _check(st, ctx=None):
    if st != NKF_OK:
        msg = load_library().nkf_last_error(ctx).decode()
        raise NkfError(st, msg)


# ------------------------------------------------------------------ contexts
_ctx_cache = {}


def _context(device, stream):
    """One library context per (device, stream); it owns the workspace."""
    key = (device, stream)
    ctx = _ctx_cache.get(key)
    if ctx is None:
        lib = load_library()
        h = ct.c_void_p()
        with torch.cuda.device(device):
            _check(lib.nkf_create(ct.byref(h), ct.c_void_p(stream)))
        ctx = h
        _ctx_cache[key] = ctx
    return ctx


def _cur_ctx(t):
    dev = t.device.index if t.device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev).cuda_stream
    return _context(dev, stream)


def release_contexts():
    lib = load_library()
    for k, c in list(_ctx_cache.items()):
        lib.nkf_destroy(c)
    _ctx_cache.clear()


# ------------------------------------------------------------------ helpers
def make_params(*, sigma_s=3.0, sigma_r=30.0, r=16, radius=-1, spatial="gaussian", guide="self",
                patch_radius=3, precision="fp32", iters=10, seed=0, tau=1e-10, center=None):
    p = Params()
    load_library().nkf_params_default(ct.byref(p))
    p.sigma_s = float(sigma_s)
    p.sigma_r = float(sigma_r)
    p.r = int(r)
    p.radius = int(radius)
    p.spatial = SPATIAL[spatial]
    p.guide = GUIDE[guide]
    p.patch_radius = int(patch_radius)
    p.prec = PREC[precision]
    p.kmeans_iters = int(iters)
    p.seed = int(seed) & ((1 << 64) - 1)
    p.eig_rel_tol = float(tau)
    p.center = float("nan") if center is None else float(center)
    return p


def _dev_f32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return ct.c_void_p(t.data_ptr())


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(0)


def _guide_dim(f, p, guide, patch_radius):
    H, W, C = f.shape
    if guide == "explicit":
        if p is None or p.dim() != 3 or p.shape[:2] != f.shape[:2]:
            raise ValueError("explicit guide needs p of shape [H, W, D]")
        return p.shape[2]
    if guide == "self":
        return C
    if guide == "patch":
        return C * (2 * patch_radius + 1) ** 2
    raise ValueError(guide)


# ------------------------------------------------------------------ API
def version():
    return load_library().nkf_version().decode()


def filter(f, p=None, *, sigma_s=3.0, sigma_r=30.0, r=16, radius=-1, spatial="gaussian",
           guide=None, patch_radius=3, precision="fp32", iters=10, seed=0, tau=1e-10, center=None,
           return_eta=False, return_r_eff=False):
    """Nystrom kernel filter g_hat of f [H, W, C] guided by p (Algorithm 1)."""
    if guide is None:
        guide = "explicit" if p is not None else "self"
    H, W, C = f.shape
    D = _guide_dim(f, p, guide, patch_radius)
    prm = make_params(sigma_s=sigma_s, sigma_r=sigma_r, r=r, radius=radius, spatial=spatial,
                      guide=guide, patch_radius=patch_radius, precision=precision, iters=iters,
                      seed=seed, tau=tau, center=center)
    out = torch.empty_like(f)
    eta = torch.empty((H, W), dtype=torch.float32, device=f.device) if return_eta else None
    reff = ct.c_int(0)
    ctx = _cur_ctx(f)
    lib = load_library()
    _check(lib.nkf_filter(ctx, H, W, C, _dev_f32(f, "f"), D,
                          _dev_f32(p, "p") if guide == "explicit" else ct.c_void_p(0),
                          ct.byref(prm), _ptr(out), _ptr(eta), ct.byref(reff)), ctx)
    res = (out,)
    if return_eta:
        res += (eta,)
    if return_r_eff:
        res += (reff.value,)
    return res[0] if len(res) == 1 else res


def patch_pca(f, *, patch_radius=3, dim=25, seed=0, return_eigvals=False):
    """PCA-reduced patch guide [H, W, dim] (float32, device) of PCA-NLM; use
    it as the explicit guide ``p`` of ``filter``."""
    H, W, C = f.shape
    g = torch.empty((H, W, dim), dtype=torch.float32, device=f.device)
    ev = np.zeros(dim, np.float64)
    ctx = _cur_ctx(f)
    _check(load_library().nkf_patch_pca(ctx, H, W, C, _dev_f32(f, "f"), patch_radius, dim, seed, _ptr(g),
                                        ev.ctypes.data_as(ct.c_void_p)), ctx)
    return (g, ev) if return_eigvals else g


def kmeans(f, p=None, *, r=16, iters=10, seed=0, guide=None, patch_radius=3, precision="fp32",
           return_labels=False, sigma_r=1.0, sigma_s=1.0):
    """k-means landmarks [r, D] (float32, device)."""
    if guide is None:
        guide = "explicit" if p is not None else "self"
    H, W, C = f.shape
    D = _guide_dim(f, p, guide, patch_radius)
    prm = make_params(sigma_s=sigma_s, sigma_r=sigma_r, r=r, guide=guide, patch_radius=patch_radius,
                      precision=precision, iters=iters, seed=seed)
    cen = torch.empty((r, D), dtype=torch.float32, device=f.device)
    lab = torch.empty((H, W), dtype=torch.int32, device=f.device) if return_labels else None
    ctx = _cur_ctx(f)
    _check(load_library().nkf_kmeans(ctx, H, W, C, _dev_f32(f, "f"), D,
                                     _dev_f32(p, "p") if guide == "explicit" else ct.c_void_p(0),
                                     ct.byref(prm), _ptr(cen), _ptr(lab)), ctx)
    return (cen, lab) if return_labels else cen


def kmeans_iterate(f, centroids, p=None, *, iters=1, guide=None, patch_radius=3, precision="fp32",
                   return_labels=False):
    """``iters`` Lloyd iterations from ``centroids`` (updated in place)."""
    if guide is None:
        guide = "explicit" if p is not None else "self"
    H, W, C = f.shape
    D = _guide_dim(f, p, guide, patch_radius)
    r = centroids.shape[0]
    prm = make_params(r=r, guide=guide, patch_radius=patch_radius, precision=precision)
    lab = torch.empty((H, W), dtype=torch.int32, device=f.device) if return_labels else None
    ctx = _cur_ctx(f)
    _check(load_library().nkf_kmeans_iterate(ctx, H, W, C, _dev_f32(f, "f"), D,
                                             _dev_f32(p, "p") if guide == "explicit" else ct.c_void_p(0),
                                             ct.byref(prm), _dev_f32(centroids, "centroids"), int(iters),
                                             _ptr(lab)), ctx)
    return (centroids, lab) if return_labels else centroids


def landmark_factor(centroids, sigma_r, tau=1e-10):
    """Host FP64 factor of the landmark Gram matrix: (Q [r, r], alpha [r]
    ascending, F [r, r_eff], r_eff) as numpy arrays."""
    c = np.ascontiguousarray(np.asarray(centroids.detach().cpu() if isinstance(centroids, torch.Tensor)
                                        else centroids, dtype=np.float64))
    r, D = c.shape
    Q = np.zeros((r, r))
    al = np.zeros(r)
    F = np.zeros((r, r))
    reff = ct.c_int(0)
    st = load_library().nkf_landmark_factor(r, D, c.ctypes.data_as(ct.c_void_p), float(sigma_r), float(tau),
                                            Q.ctypes.data_as(ct.c_void_p), al.ctypes.data_as(ct.c_void_p),
                                            F.ctypes.data_as(ct.c_void_p), ct.byref(reff))
    _check(st)
    return Q, al, np.ascontiguousarray(F[:, :reff.value]), reff.value


def filter_landmarks(f, centroids, F, p=None, *, sigma_s=3.0, sigma_r=30.0, radius=-1,
                     spatial="gaussian", guide=None, patch_radius=3, precision="fp32", center=None,
                     return_eta=False, out=None, eta=None, noalloc=False):
    """Forward pass with given landmarks [r, D] and factor F [r, r_eff]
    (float64; host or device).  noalloc=True calls the allocation-free entry
    point (the library's fixed device scratch instead of its workspace; pass
    F, out and eta as device tensors for a call that allocates nothing)."""
    if guide is None:
        guide = "explicit" if p is not None else "self"
    H, W, C = f.shape
    D = _guide_dim(f, p, guide, patch_radius)
    r = centroids.shape[0]
    if isinstance(F, torch.Tensor):
        Ft = F.to(device=f.device, dtype=torch.float64).contiguous()
    else:
        # a host factor goes through pinned memory, so the copy is queued on the
        # stream instead of blocking until the stream drains
        Fh = torch.from_numpy(np.ascontiguousarray(F, dtype=np.float64)).pin_memory()
        Ft = Fh.to(device=f.device, non_blocking=True)
    r_eff = Ft.shape[1]
    prm = make_params(sigma_s=sigma_s, sigma_r=sigma_r, r=r, radius=radius, spatial=spatial, guide=guide,
                      patch_radius=patch_radius, precision=precision, center=center)
    if out is None:
        out = torch.empty_like(f)
    if return_eta and eta is None:
        eta = torch.empty((H, W), dtype=torch.float32, device=f.device)
    ctx = _cur_ctx(f)
    lib = load_library()
    fn = lib.nkf_filter_landmarks_noalloc if noalloc else lib.nkf_filter_landmarks
    _check(fn(ctx, H, W, C, _dev_f32(f, "f"), D,
                                               _dev_f32(p, "p") if guide == "explicit" else ct.c_void_p(0),
                                               ct.byref(prm), _dev_f32(centroids, "centroids"),
                                               ct.c_void_p(Ft.data_ptr()), int(r_eff), _ptr(out),
                                               _ptr(eta if return_eta else None)), ctx)
    return (out, eta) if return_eta else out


def seed_indices(N, r, seed):
    idx = np.zeros(r, np.int64)
    _check(load_library().nkf_seed_indices(int(N), int(r), int(seed) & ((1 << 64) - 1),
                                           idx.ctypes.data_as(ct.c_void_p)))
    return idx


def spatial_taps(radius, sigma_s, spatial="gaussian"):
    S = ct.c_int(0)
    _check(load_library().nkf_spatial_taps(int(radius), float(sigma_s), SPATIAL[spatial], ct.byref(S), None))
    taps = np.zeros(2 * S.value + 1, np.float32)
    _check(load_library().nkf_spatial_taps(int(radius), float(sigma_s), SPATIAL[spatial], ct.byref(S),
                                           taps.ctypes.data_as(ct.c_void_p)))
    return S.value, taps


def enable_timing(t, enable=True):
    """Turn per-stage HIP-event timing on for the context of ``t``'s device and
    the current stream."""
    ctx = _cur_ctx(t)
    _check(load_library().nkf_enable_timing(ctx, 1 if enable else 0), ctx)


def set_conv_chunks(t, nch):
    """Row chunks per convolution tile for the context of ``t``'s device and
    the current stream (0: automatic); see nkf_set_conv_chunks."""
    ctx = _cur_ctx(t)
    _check(load_library().nkf_set_conv_chunks(ctx, int(nch)), ctx)


def enable_stats(t, enable=True):
    """Record the statistics of each forward call (r_eff, cond(A), the pixels
    that took the eta_hat <= 0 guard, min eta_hat) for the context of ``t``'s
    device and the current stream."""
    ctx = _cur_ctx(t)
    _check(load_library().nkf_enable_stats(ctx, 1 if enable else 0), ctx)


def get_stats(t):
    """The record of the last forward call (a dict; waits for the stream), or
    None if none was recorded."""
    ctx = _cur_ctx(t)
    st = Stats()
    _check(load_library().nkf_get_stats(ctx, ct.byref(st)), ctx)
    if not st.valid:
        return None
    return {k: getattr(st, k) for k, _ in Stats._fields_ if k != "valid"}


def stage_times(t, reset=True):
    """{stage: (milliseconds, intervals)} accumulated since the last reset."""
    ctx = _cur_ctx(t)
    ms = np.zeros(len(STAGES))
    cnt = np.zeros(len(STAGES), np.int32)
    _check(load_library().nkf_stage_times(ctx, ms.ctypes.data_as(ct.c_void_p), cnt.ctypes.data_as(ct.c_void_p),
                                          1 if reset else 0), ctx)
    return {s: (float(m), int(c)) for s, m, c in zip(STAGES, ms, cnt)}


def filter_backward(f, centroids, Q, alpha, r_eff, grad_out, p=None, *, sigma_s=3.0, sigma_r=30.0,
                    radius=-1, spatial="gaussian", guide=None, patch_radius=3, center=None,
                    need_f=True, need_p=True, need_sigma_r=True, need_sigma_s=True, out=None, eta=None):
    """Gradients of L with dL/dg = grad_out through the filter with given
    landmarks (held fixed).  Q [r, r] / alpha [r] are the eigenpairs returned
    by landmark_factor for the same landmarks and sigma_r.  ``out`` / ``eta``
    (optional) are the forward's output and eta_hat for the same arguments;
    given both, the forward convolutions are not repeated.  Returns
    (df, dp, dsigma_r, dsigma_s); entries not requested are None.  dp is the
    gradient w.r.t. the guide (for guide='self' add it to df)."""
    if guide is None:
        guide = "explicit" if p is not None else "self"
    H, W, C = f.shape
    D = _guide_dim(f, p, guide, patch_radius)
    r = centroids.shape[0]
    prm = make_params(sigma_s=sigma_s, sigma_r=sigma_r, r=r, radius=radius, spatial=spatial, guide=guide,
                      patch_radius=patch_radius, center=center)
    Qh = np.ascontiguousarray(np.asarray(Q, np.float64))
    ah = np.ascontiguousarray(np.asarray(alpha, np.float64))
    go = grad_out.contiguous()
    df = torch.empty_like(f) if need_f else None
    dp = torch.empty((H, W, D), dtype=torch.float32, device=f.device) if need_p else None
    dsr = ct.c_double(0.0)
    dss = ct.c_double(0.0)
    ctx = _cur_ctx(f)
    _check(load_library().nkf_filter_backward(
        ctx, H, W, C, _dev_f32(f, "f"), D, _dev_f32(p, "p") if guide == "explicit" else ct.c_void_p(0),
        ct.byref(prm), _dev_f32(centroids, "centroids"), Qh.ctypes.data_as(ct.c_void_p),
        ah.ctypes.data_as(ct.c_void_p), int(r_eff), _dev_f32(go, "grad_out"), _ptr(df), _ptr(dp),
        ct.byref(dsr) if need_sigma_r else None, ct.byref(dss) if need_sigma_s else None,
        _dev_f32(out, "out") if out is not None else ct.c_void_p(0),
        _dev_f32(eta, "eta") if eta is not None else ct.c_void_p(0)), ctx)
    return (df, dp, dsr.value if need_sigma_r else None, dss.value if need_sigma_s else None)


class NystromFilter(torch.autograd.Function):
    """Differentiable Nystrom filter with fixed landmarks.

    apply(f, p, sigma_r, sigma_s, landmarks, radius, spatial, center, tau):
    f [H, W, C] float32 CUDA; p [H, W, D] or None (the image guides itself);
    sigma_r, sigma_s 0-d float64 tensors (or floats); landmarks [r, D] float32
    CUDA.  Gradients flow to f, p, sigma_r and sigma_s; the landmarks and the
    window radius are held fixed.  The forward keeps its output and eta_hat
    (C + 1 planes); the backward recomputes the embedding instead of storing
    the r_eff (C + 1) convolution planes."""

    @staticmethod
    def forward(ctx, f, p, sigma_r, sigma_s, landmarks, radius=-1, spatial="gaussian", center=None, tau=1e-10):
        sr = float(sigma_r)
        ss = float(sigma_s)
        Q, al, F, reff = landmark_factor(landmarks, sr, tau)
        out, eta = filter_landmarks(f, landmarks, F, p, sigma_s=ss, sigma_r=sr, radius=radius, spatial=spatial,
                                    center=center, return_eta=True)
        ctx.save_for_backward(f, p if p is not None else f, landmarks, out, eta)
        ctx.self_guided = p is None
        ctx.factor = (Q, al, reff)
        ctx.cfg = dict(sigma_s=ss, sigma_r=sr, radius=radius, spatial=spatial, center=center)
        ctx.sigma_types = (sigma_r, sigma_s)
        return out

    @staticmethod
    def backward(ctx, G):
        f, p, landmarks, out, eta = ctx.saved_tensors
        Q, al, reff = ctx.factor
        need_p = ctx.self_guided or ctx.needs_input_grad[1]
        sr_t, ss_t = ctx.sigma_types
        need_sr = ctx.needs_input_grad[2]
        need_ss = ctx.needs_input_grad[3] and ctx.cfg["spatial"] == "gaussian"
        df, dp, dsr, dss = filter_backward(
            f, landmarks, Q, al, reff, G, None if ctx.self_guided else p, need_f=True, need_p=need_p,
            need_sigma_r=need_sr, need_sigma_s=need_ss, out=out, eta=eta, **ctx.cfg)
        if ctx.self_guided:
            df = df + dp
            dp = None

        def as_grad(v, like):
            if v is None or not isinstance(like, torch.Tensor):
                return None
            return torch.tensor(v, dtype=like.dtype, device=like.device)

        return (df, dp, as_grad(dsr, sr_t), as_grad(dss, ss_t), None, None, None, None, None)
