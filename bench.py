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
kernel, timed with HIP events on the stream it runs on; ``cpu_baseline`` is
the FP64 oracle on a bounded crop of the same image.
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
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


def conv_flops_per_pixel(r_eff, C, T):
    """Algorithmic flops of the convolution + contraction stage per pixel:
    P = r_eff (C+1) planes, two separable T-tap passes (2 flops per tap),
    the r_eff C products u_k f_c, the 2P contraction flops and the C
    divisions plus C offset additions."""
    P = r_eff * (C + 1)
    return 4 * P * T + r_eff * C + 2 * P + 2 * C


def conv_bytes_per_pixel(r_eff, C):
    """Compulsory HBM bytes of the stage per pixel: u read (r_eff floats),
    f read and g written (C floats each)."""
    return 4 * (r_eff + 2 * C)


def _traffic(n_launch_px):
    path = os.path.join(ROOT, "profiles", "conv_color_blf_2048_traffic.json")
    src = os.path.join(ROOT, "paper_1901_06112_amd", "csrc", "kernels_conv.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if rec.get("kernels_conv_sha256") != sha:
            return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(crop=1024):
    """The FP64 oracle (k-means + Algorithm 1) on a crop x crop centre crop
    of the workload image, single-threaded BLAS."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import kmeans, nystrom, seeding
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
    return {"value": crop * crop / dt / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{crop}x{crop} centre crop of the 2048x2048 image, full oracle path "
                      f"(seeding, {prm['iters']} Lloyd iterations, Algorithm 1 in FP64), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-crop", type=int, default=1024)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the filter has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1901_06112_amd import nkf, synth

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
    traffic = _traffic(N)
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
                     "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic, "launch_ms": round(conv_launch_ms, 4),
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_hbm_GBs": round(conv_bytes_per_pixel(r_eff, C) * N / (conv_launch_ms * 1e-3) / 1e9, 1)},
        "stages_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in st.items() if v[1] > 0},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.cpu_crop)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
