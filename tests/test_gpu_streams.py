"""Library contexts on concurrent streams and host threads (the way the
differentiation batch is scheduled): every image's forward output, eta_hat
and gradients equal, bit for bit, those of the same calls made one after
another on one stream.  The forward with given landmarks and the backward
are deterministic (fixed summation orders), so any sharing of state between
contexts would show as a difference."""
import threading

import numpy as np
import pytest
import torch

from oracle import kmeans, seeding
from paper_1901_06112_amd import synth

pytestmark = pytest.mark.gpu


def _nkf():
    from paper_1901_06112_amd import nkf
    nkf.load_library()
    return nkf


def _images():
    nkf = _nkf()
    out = []
    for i, (h, w) in enumerate([(96, 130), (141, 77), (64, 200), (120, 120)]):
        f, prm = synth.workload("diff_batch8", h, w, seed=300 + i)
        P = f.reshape(-1, 3).astype(np.float64)
        c, _, _ = kmeans.lloyd(P, P[seeding.distinct_indices(P.shape[0], 16, i)], 4)
        c32 = c.astype(np.float32)
        Q, al, F, reff = nkf.landmark_factor(c32.astype(np.float64), prm["sigma_r"])
        G = np.random.default_rng(i).normal(0, 1, f.shape).astype(np.float32)
        out.append((torch.from_numpy(f).cuda(), torch.from_numpy(c32).cuda(), Q, al, F, reff,
                    torch.from_numpy(G).cuda(), prm))
    torch.cuda.synchronize()
    return out


def _run(im):
    nkf = _nkf()
    ft, ct_, Q, al, F, reff, G, prm = im
    kw = dict(sigma_s=prm["sigma_s"], sigma_r=prm["sigma_r"], radius=prm["S"])
    out, eta = nkf.filter_landmarks(ft, ct_, F, return_eta=True, **kw)
    df, dp, dsr, dss = nkf.filter_backward(ft, ct_, Q, al, reff, G, out=out, eta=eta, **kw)
    torch.cuda.current_stream().synchronize()
    return [out.cpu().numpy(), eta.cpu().numpy(), df.cpu().numpy(), np.array([dsr, dss])]


def test_contexts_on_concurrent_streams_match_one_stream():
    imgs = _images()
    ref = [_run(im) for im in imgs]
    streams = [torch.cuda.Stream() for _ in range(2)]
    got = [None] * len(imgs)
    errors = []

    def worker(t):
        try:
            with torch.cuda.stream(streams[t]):
                for i in range(t, len(imgs), 2):
                    got[i] = _run(imgs[i])
        except BaseException as e:
            errors.append(e)

    for _ in range(2):  # twice: the second pass reuses the contexts and their workspaces
        threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        assert not errors, errors[0]
        for i in range(len(imgs)):
            for a, b in zip(got[i], ref[i]):
                assert np.array_equal(a, b), f"image {i} differs on concurrent streams"
