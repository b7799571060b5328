#!/usr/bin/env python3
"""Throughput of the Nystrom colour bilateral filter on one MI355X.

Workload (one step = one whole nkf_filter call, Algorithm 1 end to end):
a 2048 x 2048 x 3 float32 image (smooth value-noise colour field, 30 random
convex polygons, Gaussian noise sigma 25, clipped to [0, 255]; seeded), the
image as its own guide, spatial Gaussian sigma_s = 5 on a 31 x 31 window,
range sigma_r = 40, r = 32 k-means landmarks after 15 Lloyd iterations.
The step runs k-means seeding and iterations, the host FP64 landmark factor
(one device-to-host round trip), the embedding, and the 128 convolution
planes fused with the contraction and normalisation.  Inputs are resident in
HBM before the timed region.

Prints one JSON line; ``roofline`` describes the convolution + contraction
kernel, timed with HIP events on the stream it runs on (``launch_ms``), next
to the rocprofv3 average of the committed profile of the same command
(``launch_ms_rocprof``); ``cpu_baseline`` is the FP64 oracle on a bounded
crop of the same image with all host cores (Lloyd iterations in one process,
Algorithm 1 over row strips in a pool of worker processes), with the
single-core figure beside it and (``quality``) the PSNR of the GPU output
against the exact brute-force filter on the centre 256 x 256 pixels.  Each
entry of ``workloads`` carries the roofline of its convolution stage (HBM for
the box window, FP64-rate ALU for the Gaussian) and the MFMA fractions of
its 16-bit stages; the differentiation batch carries the ALU fraction of its
forward and forward + backward.  ``workloads`` holds the
other configurations, each timed the same way (whole calls, inputs resident):
the hyperspectral BLF (512 x 512 x 128, d = 128) in the plain FP32 form and
the BF16 precision form, the colour NLM (1024 x 1024, 7 x 7 x 3 patches,
d = 147, 21 x 21 box) in FP32 and FP16, the colour PCA-NLM (the same image,
patches reduced by PCA to 25 dimensions, 31 landmarks) in FP32 and FP16, and
the differentiation batch (eight 384..1024-sided images, fixed landmarks)
forward and forward + backward.
``--leg NAME`` runs one of those legs alone (for profiling).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "color_blf_2048"
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak (packed FP32)
PEAK_FP64_TFLOPS = 78.6           # MI355X FP64 vector peak: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2
PEAK_HBM_GBS = 8000.0
PEAK_MFMA16_TFLOPS = 2500.0       # MI355X dense BF16 / FP16 matrix peak


def wk_flops_per_pixel(r_eff, C, T):
    """Algorithmic flops per pixel of the windowed form (the 16-bit forms on
    C > 3): for each of the T^2 window pixels y, K_hat(x, y) = u(x).u(y)
    (2 r_eff), the weight (1) and the weighted sums of f~(y) and of 1 for
    eta_hat (2 (C + 1))."""
    return T * T * (2 * r_eff + 1 + 2 * (C + 1))


def wk_mfma_flops_issued(H, W, C, r_eff, S):
    """Matrix-core flops the windowed kernel issues per launch: 8-row by
    32-column query tiles of 8 waves, two 16-query units per wave; a wave
    works on the 2S + 5 key rows that reach one of its units: three 16-key
    tiles x r_eff / 32 steps (rounded up to 32 or 64) x three split passes x
    two units on GEMM1, and 2 x two units per 16 channels on GEMM2; each
    16x16x32 MFMA is 16384 flops.  Includes the tile halo, the padding and
    the zero half of the last key pair: the work the kernel actually
    issues, next to the algorithmic work."""
    rs = 1 if r_eff <= 32 else 2
    ct = (C + 15) // 16
    chunks = (ct + 7) // 8
    per_row = chunks * (3 * rs * 3 * 2) + ct * 2 * 2
    blocks = ((W + 31) // 32) * ((H + 7) // 8)
    return blocks * 8 * (2 * S + 5) * per_row * 16384


def conv_flops_per_pixel(r_eff, C, T):
    """Algorithmic flops of the convolution + contraction stage per pixel:
    P = r_eff (C+1) planes, two separable T-tap passes (2 flops per tap),
    the r_eff C products u_k f_c, the 2P contraction flops and the C
    divisions plus C offset additions."""
    P = r_eff * (C + 1)
    return 4 * P * T + r_eff * C + 2 * P + 2 * C


def embed_flops_per_pixel(r_eff, r, D):
    """Embedding u = F^T b: 3 flops per guide dimension and landmark for the
    distances (difference, multiply, add), one exponential per landmark
    (counted as one flop) and 2 r r_eff for the mix."""
    return 3 * D * r + r + 2 * r * r_eff


def fwd_flops_per_pixel(r_eff, r, D, C, T):
    """Forward with given landmarks: embedding + convolutions + contraction."""
    return embed_flops_per_pixel(r_eff, r, D) + conv_flops_per_pixel(r_eff, C, T)


def bwd_flops_per_pixel(r_eff, r, D, C, T):
    """Backward with the forward's output and eta given (as the autograd
    function runs it), per pixel, with P = r_eff (C + 1) planes:
    the embedding recomputed; du_dir: the P planes convolved again (4 P T) and
    combined with (beta, a) (2 P); the sigma_s pass: P planes through the w1
    and w1' row taps and the matching column taps (8 P T) and the products
    (2 P); the adjoint: P planes (4 P T), du and df (4 P); the reduction: the
    distances again (3 D r), db = F du (2 r r_eff), dp (3 D r), the sigma_r
    terms (4 r) and R = sum b du_dir^T (2 r r_eff); (beta, a): 4 C."""
    P = r_eff * (C + 1)
    return (embed_flops_per_pixel(r_eff, r, D) + (4 * P * T + 2 * P) + (8 * P * T + 2 * P)
            + (4 * P * T + 4 * P) + (6 * D * r + 4 * r + 4 * r * r_eff) + 4 * C)


def conv_bytes_per_pixel(r_eff, C):
    """Compulsory HBM bytes of the stage per pixel: u read (r_eff floats),
    f read and g written (C floats each)."""
    return 4 * (r_eff + 2 * C)


CONV_SOURCES = ("kernels_conv.hip", "conv_core.h", "device_common.h")


def conv_source_hash():
    """SHA-256 over the sources of the convolution kernel, so that a stored
    counter reading is used only for the kernel it was taken from."""
    h = hashlib.sha256()
    for name in CONV_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1901_06112_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def _traffic():
    """HBM bytes per launch of the convolution kernel from the committed
    FETCH_SIZE / WRITE_SIZE readings (already scaled by the copy-kernel
    calibration), or None when the kernel has changed since."""
    path = os.path.join(ROOT, "profiles", "conv_color_blf_2048_traffic.json")
    try:
        rec = json.load(open(path))
        if rec.get("conv_sources_sha256") != conv_source_hash():
            return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


PROFILE_HEADLINE = os.path.join("profiles", "conv_color_blf_2048.md")


def rocprof_launch_ms(kernel_prefix, path=PROFILE_HEADLINE):
    """Average duration (ms) of the kernel whose name starts with kernel_prefix
    in a committed rocprofv3 --stats summary (a markdown table with the
    average in microseconds), or None."""
    try:
        for line in open(os.path.join(ROOT, path)):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 3 and cells[0].strip("`").startswith(kernel_prefix):
                return float(cells[2]) / 1e3
    except (OSError, ValueError):
        pass
    return None


def copy_calibration(nbytes, reps):
    """Device-to-device copies of a known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: each copy reads and writes nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_workers():
    """Worker processes for the all-cores oracle: the cores this process may
    run on, at most 16 (a one-GPU share of the GPU hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_strip(args):
    """Algorithm 1 (FP64 oracle) on rows [y0, y1) of the image: the strip plus
    an S-row halo on each side, so that every window of the kept rows sees the
    same pixels as in the whole image (zero extension only at the image edge)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import nystrom
    fc, c, y0, y1, sigma_s, sigma_r, S = args
    a, b = max(0, y0 - S), min(fc.shape[0], y1 + S)
    with threadpool_limits(1):
        g = nystrom.nystrom_filter(fc[a:b], fc[a:b], c, sigma_s, sigma_r, S)
    return y0, np.ascontiguousarray(g[y0 - a:y0 - a + (y1 - y0)])


def cpu_baseline_parallel(crop=1024, workers=None):
    """The FP64 oracle on the crop x crop centre crop with all host cores: the
    Lloyd iterations in one process (NumPy, BLAS threads = all cores), then
    Algorithm 1 over horizontal strips in a pool of worker processes (the
    strips' outputs equal the whole-image output exactly).  Run before the GPU
    is initialised (the pool is forked)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import kmeans, seeding
    from paper_1901_06112_amd import synth

    workers = workers or cpu_workers()
    f, prm = synth.workload(WORKLOAD)
    y0 = (f.shape[0] - crop) // 2
    fc = np.ascontiguousarray(f[y0:y0 + crop, y0:y0 + crop]).astype(np.float64)
    nstrip = 4 * workers
    bounds = [(crop * i // nstrip, crop * (i + 1) // nstrip) for i in range(nstrip)]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        P = fc.reshape(-1, 3)
        c0 = P[seeding.distinct_indices(P.shape[0], prm["r"], prm["landmark_seed"])]
        c, _, _ = kmeans.lloyd(P, c0, prm["iters"])
        t1 = time.perf_counter()
        parts = pool.map(_oracle_strip, [(fc, c, a, b, prm["sigma_s"], prm["sigma_r"], prm["S"])
                                         for a, b in bounds])
        t2 = time.perf_counter()
    assert sum(p[1].shape[0] for p in parts) == crop
    return {"value": crop * crop / (t2 - t0) / 1e6, "cores": workers, "seconds": round(t2 - t0, 2),
            "kmeans_s": round(t1 - t0, 2), "filter_s": round(t2 - t1, 2),
            "sample": f"{crop}x{crop} centre crop: {prm['iters']} Lloyd iterations in one process, then "
                      f"Algorithm 1 in FP64 over {nstrip} row strips (S-row halos) on {workers} worker processes"}


def cpu_baseline(crop=1024, gpu_out=None, gpu_landmarks=None, qcrop=256):
    """The FP64 oracle (k-means + Algorithm 1) on a crop x crop centre crop
    of the workload image, single-threaded BLAS.  With the GPU output of the
    full image and its landmarks, also the quality the throughput is quoted
    at: PSNR against the exact brute-force filter (Eq. (num)) on the centre
    qcrop x qcrop pixels, evaluated on a crop with an S-pixel margin so that
    every window lies inside it, for the GPU output and for the FP64 oracle
    with the same landmarks (the two differ by arithmetic only)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import exact, kmeans, nystrom, seeding
    from paper_1901_06112_amd import synth

    f, prm = synth.workload(WORKLOAD)
    y0 = (f.shape[0] - crop) // 2
    fc = np.ascontiguousarray(f[y0:y0 + crop, y0:y0 + crop]).astype(np.float64)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        P = fc.reshape(-1, 3)
        c0 = P[seeding.distinct_indices(P.shape[0], prm["r"], prm["landmark_seed"])]
        c, _, _ = kmeans.lloyd(P, c0, prm["iters"])
        nystrom.nystrom_filter(fc, fc, c, prm["sigma_s"], prm["sigma_r"], prm["S"])
        dt = time.perf_counter() - t0
    res = {"value": crop * crop / dt / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{crop}x{crop} centre crop of the 2048x2048 image, full oracle path "
                     f"(seeding, {prm['iters']} Lloyd iterations, Algorithm 1 in FP64), one core, {dt:.1f} s"}
    if gpu_out is not None:
        m, q = prm["S"], qcrop
        yq = (f.shape[0] - q) // 2
        fe = np.ascontiguousarray(f[yq - m:yq + q + m, yq - m:yq + q + m]).astype(np.float64)
        ex = exact.exact_filter(fe, fe, prm["sigma_s"], prm["sigma_r"], prm["S"])[m:m + q, m:m + q]
        gq = gpu_out[yq:yq + q, yq:yq + q]
        qual = {"gpu_psnr_vs_exact_dB": round(float(exact.psnr(gq, ex)), 2)}
        if gpu_landmarks is not None:
            ny = nystrom.nystrom_filter(fe, fe, gpu_landmarks, prm["sigma_s"], prm["sigma_r"], prm["S"])[m:m + q, m:m + q]
            qual["oracle_same_landmarks_psnr_vs_exact_dB"] = round(float(exact.psnr(ny, ex)), 2)
            qual["max_abs_gpu_vs_oracle"] = float(np.abs(gq - ny).max())
        qual["sample"] = (f"centre {q}x{q} pixels of the full-image GPU call; exact brute-force BLF "
                          f"({2 * m + 1}x{2 * m + 1} window); oracle: Algorithm 1 in FP64 with the GPU's landmarks")
        res["quality"] = qual
    return res


def _timed(fn, steps, warmup, timing_tensor=None):
    import torch

    from paper_1901_06112_amd import nkf
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if timing_tensor is not None:
        nkf.enable_timing(timing_tensor, True)
        nkf.stage_times(timing_tensor, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    st = None
    if timing_tensor is not None:
        st = nkf.stage_times(timing_tensor, reset=True)
        nkf.enable_timing(timing_tensor, False)
        st = {k: round(v[0] / steps, 4) for k, v in st.items() if v[1] > 0}
    return ms, st, res


def _psnr(a, b, peak):
    import torch
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * __import__("math").log10(peak * peak / mse)


def leg_precision(name, steps, warmup):
    """Plain FP32 form against the 16-bit precision form on one high-d workload.
    MFMA fractions count the algorithmic GEMM flops of the stage: 2 d r per
    pixel per Lloyd iteration (assignment) and 2 d r + 2 r r_eff per pixel
    (embedding), against the dense 16-bit MFMA peak."""
    import torch

    from paper_1901_06112_amd import nkf, synth
    f, prm = synth.workload(name)
    H, W, C = f.shape
    N = H * W
    ft = torch.from_numpy(f).cuda()
    if name.startswith("hyper"):
        kw = dict(sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], r=prm["r"], radius=prm["S"],
                  iters=prm["iters"], seed=prm["landmark_seed"])
        D, peak, forms = C, 1.0, ("fp32", "bf16")
    else:
        kw = dict(sigma_s=1.0, sigma_r=prm["sigma_r"], r=prm["r"], radius=prm["S"], spatial="box",
                  guide="patch", patch_radius=prm["patch_radius"], iters=prm["iters"],
                  seed=prm["landmark_seed"])
        D, peak, forms = C * (2 * prm["patch_radius"] + 1) ** 2, 255.0, ("fp32", "fp16")
    out = {"H": H, "W": W, "C": C, "d": D, "r": prm["r"], "S": prm["S"],
           "spatial": kw.get("spatial", "gaussian"), "kmeans_iters": prm["iters"]}
    res = {}
    for prec in forms:
        ms, st, (g, r_eff) = _timed(lambda: nkf.filter(ft, precision=prec, return_r_eff=True, **kw),
                                    steps, warmup, ft)
        ent = {"ms_per_call": round(ms, 3), "Mpixel_s": round(N / ms / 1e3, 2), "r_eff": r_eff,
               "stages_ms": st}
        conv_s = st["conv"] * 1e-3
        if kw.get("spatial") == "box":
            # box conv: HBM-bound; compulsory bytes = the embedding planes (FP64
            # in the plain form, FP32 in the 16-bit form), f read, g written
            ub = 8 if prec == "fp32" else 4
            nbytes = N * (r_eff * ub + 8 * C)
            ent["conv_roofline"] = {"kernel": "box_kernel", "bound": "hbm", "unit": "GB/s",
                                    "achieved": round(nbytes / conv_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                                    "frac": round(nbytes / conv_s / 1e9 / PEAK_HBM_GBS, 4),
                                    "algorithmic_bytes_per_launch": nbytes}
        elif prec != "fp32" and C > 3 and r_eff <= 64:
            # the windowed form on the matrix cores (stage time includes its
            # two operand-preparation kernels)
            T = 2 * prm["S"] + 1
            fl = wk_flops_per_pixel(r_eff, C, T) * N
            issued = wk_mfma_flops_issued(H, W, C, r_eff, prm["S"])
            ent["conv_roofline"] = {"kernel": "wk_kernel (windowed K_hat on MFMA)", "bound": "mfma",
                                    "unit": "TFLOP/s", "achieved": round(fl / conv_s / 1e12, 2),
                                    "peak": PEAK_MFMA16_TFLOPS,
                                    "frac": round(fl / conv_s / 1e12 / PEAK_MFMA16_TFLOPS, 4),
                                    "algorithmic_flops_per_launch": fl,
                                    "issued_mfma_flops_per_launch": issued,
                                    "issued_frac": round(issued / conv_s / 1e12 / PEAK_MFMA16_TFLOPS, 4),
                                    "fir_flops_replaced": conv_flops_per_pixel(r_eff, C, T) * N}
        else:
            T = 2 * prm["S"] + 1
            fl = conv_flops_per_pixel(r_eff, C, T) * N
            ent["conv_roofline"] = {"kernel": "conv_kernel", "bound": "alu", "unit": "TFLOP/s",
                                    "achieved": round(fl / conv_s / 1e12, 2), "peak": PEAK_FP64_TFLOPS,
                                    "frac": round(fl / conv_s / 1e12 / PEAK_FP64_TFLOPS, 4),
                                    "algorithmic_flops_per_launch": fl}
        if prec != "fp32":
            km = prm["iters"] * N * 2.0 * D * prm["r"] / (st["kmeans"] * 1e-3) / 1e12
            em = N * (2.0 * D * prm["r"] + 2.0 * prm["r"] * r_eff) / (st["embed"] * 1e-3) / 1e12
            ent["kmeans_mfma_TFLOPs"] = round(km, 2)
            ent["kmeans_mfma_frac"] = round(km / PEAK_MFMA16_TFLOPS, 4)
            ent["embed_mfma_TFLOPs"] = round(em, 2)
            ent["embed_mfma_frac"] = round(em / PEAK_MFMA16_TFLOPS, 4)
        res[prec] = (ent, g)
    out.update({p: e for p, (e, _) in res.items()})
    lo = forms[1]
    out[f"{lo}_speedup_over_fp32"] = round(res["fp32"][0]["ms_per_call"] / res[lo][0]["ms_per_call"], 3)
    out[f"psnr_{lo}_vs_fp32_dB"] = round(_psnr(res[lo][1], res["fp32"][1], peak), 2)
    return out


def leg_pca_nlm(steps, warmup):
    """Colour PCA-NLM (the paper's NLM): the NLM image, 7x7x3 patches reduced
    by PCA to 25 dimensions (nkf_patch_pca), 21x21 box, 31 landmarks, sigma_r =
    3 x the noise level.  One call = PCA guide + filter with the reduced
    explicit guide, in the FP32 form and the FP16 form."""
    import numpy as np
    import torch

    from paper_1901_06112_amd import nkf, synth
    f, prm = synth.workload("color_pca_nlm_1024")
    H, W, C = f.shape
    N = H * W
    ft = torch.from_numpy(f).cuda()
    pk = dict(patch_radius=prm["patch_radius"], dim=prm["pca_dim"], seed=prm["seed"])
    kw = dict(sigma_s=1.0, sigma_r=prm["sigma_r"], r=prm["r"], radius=prm["S"], spatial="box",
              iters=prm["iters"], seed=prm["landmark_seed"])
    pca_ms, _, _ = _timed(lambda: nkf.patch_pca(ft, **pk), steps, warmup)
    out = {"H": H, "W": W, "C": C, "d_patch": C * (2 * prm["patch_radius"] + 1) ** 2, "d_pca": prm["pca_dim"],
           "r": prm["r"], "S": prm["S"], "spatial": "box", "sigma_r": prm["sigma_r"], "kmeans_iters": prm["iters"],
           "pca_ms": round(pca_ms, 3)}
    res = {}
    for prec in ("fp32", "fp16"):
        def call():
            g = nkf.patch_pca(ft, **pk)
            return nkf.filter(ft, g, precision=prec, return_r_eff=True, **kw)
        ms, st, (g, r_eff) = _timed(call, steps, warmup, ft)
        nbytes = N * (r_eff * (8 if prec == "fp32" else 4) + 8 * C)
        conv_s = st["conv"] * 1e-3
        res[prec] = ({"ms_per_call": round(ms, 3), "Mpixel_s": round(N / ms / 1e3, 2), "r_eff": r_eff,
                      "stages_ms": st,
                      "conv_roofline": {"kernel": "box_kernel", "bound": "hbm", "unit": "GB/s",
                                        "achieved": round(nbytes / conv_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                                        "frac": round(nbytes / conv_s / 1e9 / PEAK_HBM_GBS, 4),
                                        "algorithmic_bytes_per_launch": nbytes}}, g)
    out.update({p: e for p, (e, _) in res.items()})
    # each form runs its own k-means, which in 25 dimensions may settle on other
    # landmarks; the arithmetic of the two forms is compared with shared ones
    g = nkf.patch_pca(ft, **pk)
    cen = nkf.kmeans(ft, g, r=prm["r"], iters=prm["iters"], seed=prm["landmark_seed"])
    Q, al, F, r_eff = nkf.landmark_factor(cen.cpu().numpy().astype(np.float64), prm["sigma_r"])
    fl = {prec: nkf.filter_landmarks(ft, cen, F, g, sigma_s=1.0, sigma_r=prm["sigma_r"], radius=prm["S"],
                                     spatial="box", precision=prec, return_eta=True) for prec in ("fp32", "fp16")}
    # supported pixels: eta_hat keeps >= 1e-3 of the exact filter's least mass
    # there (the pixel's own term, w(0) = 1 for the box); elsewhere no
    # landmark is near the pixel's guide value and 1 / eta_hat amplifies
    # any rounding, the FP64 result's included
    sup = fl["fp32"][1] >= 1e-3
    out["psnr_fp16_vs_fp32_same_landmarks_dB"] = round(_psnr(fl["fp16"][0], fl["fp32"][0], 255.0), 2)
    out["psnr_fp16_vs_fp32_same_landmarks_supported_dB"] = round(
        _psnr(fl["fp16"][0][sup], fl["fp32"][0][sup], 255.0), 2)
    out["unsupported_pixels"] = int((~sup).sum().item())
    out["psnr_fp16_vs_fp32_own_landmarks_dB"] = round(_psnr(res["fp16"][1], res["fp32"][1], 255.0), 2)
    return out


def _on_streams(imgs, fn, streams):
    """fn(img) for every image, image i on stream i mod len(streams) from its
    own host thread (a library context per stream, created on first use; the
    library's calls release the interpreter lock), so the small images of a
    batch overlap on the GPU and one image's host finish of the sigma
    gradients overlaps the others' work."""
    import threading

    import torch
    nst = len(streams)
    errors = []

    def worker(t):
        try:
            with torch.cuda.stream(streams[t]):
                for i in range(t, len(imgs), nst):
                    fn(imgs[i])
        except BaseException as e:  # re-raised on the calling thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(nst)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]


def leg_diff(steps, warmup, nstreams=4):
    """Differentiation batch: eight images, landmarks fixed (k-means outside the
    timed region), forward and forward + hand-written backward (df, dp,
    d sigma_r, d sigma_s): one call per image, the images spread over
    `nstreams` streams (the one-stream figures beside them)."""
    import numpy as np
    import torch

    from paper_1901_06112_amd import nkf, synth
    sizes = synth.batch_sizes()
    imgs = []
    for i, (h, w) in enumerate(sizes):
        f, prm = synth.workload("diff_batch8", h, w, seed=1050 + i)
        ft = torch.from_numpy(f).cuda()
        c = nkf.kmeans(ft, r=prm["r"], iters=prm["iters"], seed=prm["landmark_seed"])
        Q, al, F, reff = nkf.landmark_factor(c.cpu().numpy().astype(np.float64), prm["sigma_r"])
        G = torch.from_numpy(np.random.default_rng(1050 + i).normal(0, 1, f.shape).astype(np.float32)).cuda()
        # the landmarks are fixed, so their factor stays on the device
        imgs.append((ft, c, Q, al, torch.from_numpy(F).cuda(), reff, G))
    kw = dict(sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], radius=prm["S"])
    npx = sum(h * w for h, w in sizes)

    def fwd_img(im):
        ft, c, Q, al, F, reff, G = im
        nkf.filter_landmarks(ft, c, F, **kw)

    def fwdbwd_img(im):
        # as the autograd function runs it: the backward reuses the forward's
        # output and eta_hat, and recomputes the embedding
        ft, c, Q, al, F, reff, G = im
        out, eta = nkf.filter_landmarks(ft, c, F, return_eta=True, **kw)
        nkf.filter_backward(ft, c, Q, al, reff, G, out=out, eta=eta, **kw)

    ms_f1, _, _ = _timed(lambda: [fwd_img(im) for im in imgs], steps, warmup)
    ms_b1, _, _ = _timed(lambda: [fwdbwd_img(im) for im in imgs], steps, warmup)
    streams = [torch.cuda.Stream() for _ in range(nstreams)]  # default priority
    stream_error = None
    try:
        ms_f, _, _ = _timed(lambda: _on_streams(imgs, fwd_img, streams), steps, warmup)
        ms_b, _, _ = _timed(lambda: _on_streams(imgs, fwdbwd_img, streams), steps, warmup)
    except Exception as e:  # reported in the line; the one-stream figures stand
        torch.cuda.synchronize()
        stream_error = f"{type(e).__name__}: {e}"
        ms_f, ms_b, nstreams = ms_f1, ms_b1, 1
    T = 2 * prm["S"] + 1
    fl_f = sum(fwd_flops_per_pixel(im[5], prm["r"], 3, 3, T) * im[0].shape[0] * im[0].shape[1] for im in imgs)
    fl_fb = fl_f + sum(bwd_flops_per_pixel(im[5], prm["r"], 3, 3, T) * im[0].shape[0] * im[0].shape[1]
                       for im in imgs)
    return {"images": [list(s) for s in sizes], "pixels": npx, "r": prm["r"], "S": prm["S"],
            "streams": nstreams,
            "fwd_ms": round(ms_f, 3), "fwd_Mpixel_s": round(npx / ms_f / 1e3, 2),
            "fwd_bwd_ms": round(ms_b, 3), "fwd_bwd_Mpixel_s": round(npx / ms_b / 1e3, 2),
            "one_stream": {"fwd_ms": round(ms_f1, 3), "fwd_bwd_ms": round(ms_b1, 3)},
            "stream_error": stream_error,
            "roofline": {"bound": "alu", "unit": "TFLOP/s", "peak": PEAK_FP64_TFLOPS,
                         "fwd_achieved": round(fl_f / (ms_f * 1e-3) / 1e12, 2),
                         "fwd_frac": round(fl_f / (ms_f * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                         "fwd_bwd_achieved": round(fl_fb / (ms_b * 1e-3) / 1e12, 2),
                         "fwd_bwd_frac": round(fl_fb / (ms_b * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                         "algorithmic_flops": {"fwd": fl_f, "fwd_bwd": fl_fb}}}


def leg_recursive(steps, warmup):
    """The colour BLF workload (2048^2 x 3, r = 32, sigma_r = 40, 15
    iterations) with Young and van Vliet's recursive Gaussian in place of the
    truncated window, at sigma_s = 5 (the truncated window's 31 x 31) and at
    sigma_s = 20, where no truncated window here reaches (radius <= 16): the
    recursive filter's work does not depend on sigma_s.  The conv stage's
    roofline counts the bytes its passes must move: per pixel and embedding
    plane u_k, the column pass reads u_k twice and writes the C + 1 filtered
    planes once, the row pass reads them twice and writes them once, the
    contraction reads them and u_k once (12 + 20 (C + 1) bytes), plus f read
    and g written once; the kept chunk states (about 1.1 (C + 1) bytes each
    way) are not counted."""
    import numpy as np
    import torch

    from paper_1901_06112_amd import nkf, synth
    f, prm = synth.workload("color_blf_2048")
    H, W, C = f.shape
    N = H * W
    ft = torch.from_numpy(f).cuda()
    out = {"H": H, "W": W, "C": C, "r": prm["r"], "sigma_r": prm["sigma_r"], "kmeans_iters": prm["iters"]}
    gs = {}
    for ss in (5.0, 20.0):
        kw = dict(sigma_s=ss, sigma_r=prm["sigma_r"], r=prm["r"], iters=prm["iters"], seed=prm["landmark_seed"],
                  spatial="recursive")
        ms, st, (g, r_eff) = _timed(lambda: nkf.filter(ft, return_r_eff=True, **kw), steps, warmup, ft)
        conv_s = st["conv"] * 1e-3
        nbytes = N * (r_eff * (12 + 20 * (C + 1)) + 8 * C)
        out[f"sigma_s_{ss:g}"] = {
            "ms_per_call": round(ms, 3), "Mpixel_s": round(N / ms / 1e3, 2), "r_eff": r_eff, "stages_ms": st,
            "conv_roofline": {"kernel": "rec_cols + rec_rows + rec_contract", "bound": "hbm", "unit": "GB/s",
                              "achieved": round(nbytes / conv_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                              "frac": round(nbytes / conv_s / 1e9 / PEAK_HBM_GBS, 4),
                              "algorithmic_bytes_per_launch": nbytes}}
        gs[ss] = g
    kw = dict(sigma_s=5.0, sigma_r=prm["sigma_r"], r=prm["r"], radius=prm["S"], iters=prm["iters"],
              seed=prm["landmark_seed"])
    g_fir = nkf.filter(ft, **kw)
    out["psnr_recursive_vs_truncated_sigma5_dB"] = round(_psnr(gs[5.0], g_fir, 255.0), 2)
    # forward + backward (df, dp, dsigma_r) with the landmarks fixed, as the
    # autograd function runs it, against the truncated 31 x 31 window's
    c = nkf.kmeans(ft, r=prm["r"], iters=prm["iters"], seed=prm["landmark_seed"])
    Q, al, F, reff = nkf.landmark_factor(c.cpu().numpy().astype(np.float64), prm["sigma_r"])
    Fd = torch.from_numpy(F).cuda()
    G = torch.from_numpy(np.random.default_rng(7).normal(0, 1, f.shape).astype(np.float32)).cuda()
    for name, kwb in (("recursive", dict(sigma_s=5.0, sigma_r=prm["sigma_r"], spatial="recursive")),
                      ("truncated", dict(sigma_s=5.0, sigma_r=prm["sigma_r"], radius=prm["S"]))):
        def fb():
            o, e = nkf.filter_landmarks(ft, c, Fd, return_eta=True, **kwb)
            nkf.filter_backward(ft, c, Q, al, reff, G, out=o, eta=e, need_sigma_s=False, **kwb)
        ms, _, _ = _timed(fb, steps, warmup)
        out[f"fwd_bwd_{name}_sigma5"] = {"ms": round(ms, 3), "Mpixel_s": round(N / ms / 1e3, 2),
                                         "grads": "df, dp (self guide), dsigma_r"}
    return out


LEGS = {
    "hyperspectral": lambda s, w: leg_precision("hyperspectral_512x128", s, w),
    "nlm": lambda s, w: leg_precision("color_nlm_1024", s, w),
    "diff_batch": lambda s, w: leg_diff(s, w),
    "pca_nlm": lambda s, w: leg_pca_nlm(s, w),
    "recursive": lambda s, w: leg_recursive(s, w),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-crop", type=int, default=1024)
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--leg", choices=sorted(LEGS), help="run one other workload only")
    ap.add_argument("--leg-steps", type=int, default=5)
    ap.add_argument("--copy-calibration", type=int, metavar="BYTES",
                    help="only run device copies of BYTES bytes (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the filter has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # the all-cores oracle runs first: its worker pool is forked before the GPU
    # is initialised
    par = None
    if not (a.no_cpu_baseline or a.copy_calibration or a.leg):
        par = cpu_baseline_parallel(a.cpu_crop)

    import torch

    from paper_1901_06112_amd import nkf, synth

    if a.copy_calibration:
        copy_calibration(a.copy_calibration, 5)
        return
    if a.leg:
        print(json.dumps({"leg": a.leg, **LEGS[a.leg](a.leg_steps, 1)}), flush=True)
        return

    f, prm = synth.workload(WORKLOAD)
    H, W, C = f.shape
    N = H * W
    dev = torch.device("cuda:0")
    ft = torch.from_numpy(f).to(dev)
    kw = dict(sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], r=prm["r"], radius=prm["S"],
              iters=prm["iters"], seed=prm["landmark_seed"])

    def step():
        return nkf.filter(ft, return_r_eff=True, **kw)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    nkf.enable_timing(ft, True)
    nkf.stage_times(ft, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        out, r_eff = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = nkf.stage_times(ft, reset=True)
    nkf.enable_timing(ft, False)
    assert torch.isfinite(out).all()

    ms_step = (t1 - t0) / a.steps * 1e3
    value = N / (ms_step * 1e-3) / 1e6
    T = 2 * prm["S"] + 1
    conv_ms, conv_n = st["conv"]
    conv_launch_ms = conv_ms / max(conv_n, 1)
    flops = conv_flops_per_pixel(r_eff, C, T) * N
    achieved = flops / (conv_launch_ms * 1e-3) / 1e12
    traffic = _traffic()
    conv_rocprof_ms = rocprof_launch_ms("void nkf::conv::conv_kernel<15, 4, true, 32, 0, 512, false>")
    line = {
        "metric": "Mpixel/s Nystrom BLF forward (k-means + factor + embedding + r(C+1) convolutions + "
                  "contraction), FP32",
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "H": H, "W": W, "C": C, "guide": "self", "r": prm["r"],
                   "r_eff": r_eff, "S": prm["S"], "window": T, "sigma_s": prm["sigma_s"],
                   "sigma_r": prm["sigma_r"], "kmeans_iters": prm["iters"], "spatial": "gaussian"},
        "roofline": {"kernel": "conv_kernel (convolutions + contraction + normalisation)",
                     "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "peak_basis": "FP64 vector FMA rate: the FIR passes, the kernel's dominant work, "
                                   "accumulate in FP64",
                     "frac_of_fp32_vector_peak": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic, "launch_ms": round(conv_launch_ms, 4),
                     "launch_ms_rocprof": conv_rocprof_ms,
                     "frac_rocprof": (round(flops / (conv_rocprof_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)
                                      if conv_rocprof_ms else None),
                     "sources": {"launch_ms": "HIP events around each launch on the library's stream, "
                                              "averaged over the timed steps of this run",
                                 "launch_ms_rocprof": f"{PROFILE_HEADLINE}: rocprofv3 --kernel-trace --stats "
                                                      "average of the same command (committed run)"},
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_hbm_GBs": round(conv_bytes_per_pixel(r_eff, C) * N / (conv_launch_ms * 1e-3) / 1e9, 1)},
        "stages_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in st.items() if v[1] > 0},
    }
    if not a.no_extra:
        line["workloads"] = {k: fn(a.leg_steps, 1) for k, fn in LEGS.items()}
    if not a.no_cpu_baseline:
        cen = nkf.kmeans(ft, r=prm["r"], iters=prm["iters"], seed=prm["landmark_seed"])
        one = cpu_baseline(a.cpu_crop, out.cpu().numpy().astype(np.float64),
                           cen.cpu().numpy().astype(np.float64))
        line["cpu_baseline"] = {"value": round(par["value"], 4), "unit": "Mpixel/s", "cores": par["cores"],
                                "kind": "oracle", "cpu_model": one["cpu_model"],
                                "host_cpus": os.cpu_count(), "sample": par["sample"],
                                "seconds": par["seconds"], "kmeans_s": par["kmeans_s"],
                                "filter_s": par["filter_s"],
                                "single_core": {"value": round(one["value"], 4), "cores": 1,
                                                "sample": one["sample"]},
                                "quality": one["quality"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
