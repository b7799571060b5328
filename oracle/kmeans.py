"""Lloyd's k-means on the range list.  Test infrastructure only.

Section III: the landmarks are the centroids of a partition of the range list
R = {p(x) : x in Omega} (a list: each pixel counts once, repeats included) into
m0 clusters.  The paper gives no stopping rule; this oracle runs a fixed
number of Lloyd iterations.  Readings for what the paper leaves open:
ties go to the lowest cluster index, and an empty cluster keeps its previous
centroid.  Distances are direct differences in float64.
"""
from __future__ import annotations

import numpy as np


def assign(P, c, chunk=65536):
    """Nearest-centroid labels and the squared distance to that centroid.
    ``P`` is [N, D], ``c`` is [r, D]."""
    P = np.asarray(P, np.float64)
    c = np.asarray(c, np.float64)
    N = P.shape[0]
    lab = np.empty(N, np.int64)
    dmin = np.empty(N)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        d2 = np.zeros((b - a, c.shape[0]))
        for k in range(c.shape[0]):
            diff = P[a:b] - c[k]
            d2[:, k] = np.einsum("ij,ij->i", diff, diff)
        lab[a:b] = np.argmin(d2, axis=1)  # first minimum = lowest index on ties
        dmin[a:b] = d2[np.arange(b - a), lab[a:b]]
    return lab, dmin


def update(P, lab, c_prev):
    """Cluster means; an empty cluster keeps its previous centroid."""
    P = np.asarray(P, np.float64)
    r, D = c_prev.shape
    sums = np.zeros((r, D))
    np.add.at(sums, lab, P)
    cnt = np.bincount(lab, minlength=r).astype(np.float64)
    c = np.array(c_prev, np.float64, copy=True)
    nz = cnt > 0
    c[nz] = sums[nz] / cnt[nz, None]
    return c, sums, cnt


def lloyd(P, c0, iters):
    """``iters`` Lloyd iterations from ``c0``.  Returns (centroids, labels of
    the last assignment, quantization error e of Section III before each
    update, i.e. sum of squared distances to the assigned centroid)."""
    c = np.array(c0, np.float64, copy=True)
    errs = []
    lab = None
    for _ in range(iters):
        lab, dmin = assign(P, c)
        errs.append(float(dmin.sum()))
        c, _, _ = update(P, lab, c)
    return c, lab, errs


def quantization_error(P, c):
    """e = sum_i min_j |r_i - mu_j|^2 (Section III)."""
    _, dmin = assign(P, c)
    return float(dmin.sum())
