"""Principal-component patch guide of PCA-NLM.  Test infrastructure only.

Section IV: the NLM experiments use PCA-NLM, where the collection of patches
((2pr+1)^2 n values per pixel, rho = 3 * 7^2 = 147 for colour patches of
radius 3) is reduced by PCA before the range kernel is applied, to 25 (or 6)
dimensions.  The paper names the method and the target dimension only.

Readings used here:
* the basis is estimated from the patches of a seeded sample of
  n_s = min(N, 65536) pixels, drawn with the landmark seeding's generator
  (SplitMix64 + partial Fisher-Yates, ``oracle.seeding``); all pixels when
  N <= 65536 (in index order);
* the covariance is mean-centred with 1/n_s normalisation, in FP64;
* the basis is the ``dim`` eigenvectors of the largest eigenvalues, in
  descending eigenvalue order;
* each basis vector's entry of largest magnitude is made positive (the first
  such entry on ties), which fixes the otherwise arbitrary signs;
* the guide is the centred projection g(x)_k = (p(x) - mean) . v_k.
Distances between guide values, the only thing the filter uses, do not
depend on the centring or on the signs.
"""
from __future__ import annotations

import numpy as np

from .exact import patch_guide
from .seeding import distinct_indices

SAMPLE_MAX = 65536


def sample_indices(N, seed, n_max=SAMPLE_MAX):
    """Pixels whose patches estimate the basis."""
    if N <= n_max:
        return np.arange(N, dtype=np.int64)
    return distinct_indices(N, n_max, seed)


def patch_pca(f, pr, dim, seed=0, n_max=SAMPLE_MAX):
    """(mean [D], basis V [D, dim], eigenvalues [dim] descending) of the
    patch covariance over the sample."""
    f = np.asarray(f, np.float64)
    H, W, C = f.shape
    P = patch_guide(f, pr).reshape(H * W, -1)
    S = P[sample_indices(H * W, seed, n_max)]
    mu = S.mean(axis=0)
    X = S - mu
    cov = X.T @ X / S.shape[0]
    lam, V = np.linalg.eigh(cov)
    order = np.argsort(-lam, kind="stable")[:dim]
    lam, V = lam[order], V[:, order].copy()
    for k in range(dim):
        j = int(np.argmax(np.abs(V[:, k])))
        if V[j, k] < 0:
            V[:, k] = -V[:, k]
    return mu, V, lam


def pca_guide(f, pr, dim, seed=0, n_max=SAMPLE_MAX):
    """The projected patch guide [H, W, dim] and the kept eigenvalues."""
    f = np.asarray(f, np.float64)
    H, W, C = f.shape
    mu, V, lam = patch_pca(f, pr, dim, seed, n_max)
    P = patch_guide(f, pr).reshape(H * W, -1)
    return ((P - mu) @ V).reshape(H, W, dim), lam
