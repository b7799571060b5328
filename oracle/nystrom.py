"""Nystrom fast kernel filter in the paper's own form.  Test infrastructure only.

Section III: the range kernel k(p(x), p(y)) of Eq. (num1) is replaced by
its Nystrom approximation built from r landmarks mu_1..mu_r (k-means
centroids, see ``oracle.kmeans``).  The landmark Gram matrix A (Eq. (defA))
is decomposed as A = sum_k alpha_k w_k w_k^T (Eq. (eigA)); the eigenvectors
extend to every guide value through the cross kernel B (Eq. (defB)) as
v_k = B^T w_k / alpha_k (Eq. (vk)), and K_hat = sum_k alpha_k v_k v_k^T
(Eq. (hatK)).  With that kernel the filter becomes a sum over k of spatial
convolutions of v_k f and v_k (Eqs. (finalnum), (finalden)).

Readings where the paper is silent:
* eigenvalues alpha_k <= tau * max(alpha) (tau = 1e-10) are dropped, which
  makes the rank-deficient case (coincident landmarks, sigma_r -> inf) a
  pseudo-inverse;
* pixels where eta_hat <= 0 or is not finite output f(x);
* convolutions use zero extension at the image border, as the exact filter.
"""
from __future__ import annotations

import numpy as np

from .exact import range_kernel_sqdist, spatial_taps
from .recursive import recursive_gauss_2d

DEFAULT_TAU = 1e-10


def sqdist(X, Y):
    """Pairwise squared distances by direct differences; X [n, D], Y [m, D]."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    out = np.empty((X.shape[0], Y.shape[0]))
    for j in range(Y.shape[0]):
        diff = X - Y[j]
        out[:, j] = np.einsum("ij,ij->i", diff, diff)
    return out


def landmark_gram(c, sigma_r):
    """A of Eq. (defA)."""
    return range_kernel_sqdist(sqdist(c, c), sigma_r)


def landmark_eig(c, sigma_r, tau=DEFAULT_TAU):
    """Eigenpairs of A (Eq. (eigA)) that are kept: alpha > tau * max alpha.
    Returns (alpha [r_eff], W [r, r_eff]) with alpha ascending."""
    A = landmark_gram(c, sigma_r)
    alpha, Wv = np.linalg.eigh(A)
    keep = alpha > tau * alpha.max()
    return alpha[keep], Wv[:, keep]


def cross_kernel_sr(c, P, sigma_r):
    """B^T of Eq. (defB) as an [N, r] array: entry (x, i) = k(mu_i, p(x))."""
    return range_kernel_sqdist(sqdist(P, c), sigma_r)


def extrapolated_eigvecs(c, P, sigma_r, tau=DEFAULT_TAU):
    """alpha_k and v_k = B^T w_k / alpha_k (Eq. (vk)) for the kept k; v as [N, r_eff]."""
    alpha, Wv = landmark_eig(c, sigma_r, tau)
    Bt = cross_kernel_sr(c, P, sigma_r)
    return alpha, (Bt @ Wv) / alpha[None, :]


def conv_zero(img, w1):
    """(w * img) for the separable kernel w(z) = w1(z1) w1(z2) on the square
    window, with the window intersected with the image (zero extension).
    ``img`` is [H, W] or [H, W, C]; ``w1`` is symmetric so correlation and
    convolution coincide."""
    img = np.asarray(img, np.float64)
    S = (len(w1) - 1) // 2
    H, W = img.shape[:2]
    tmp = np.zeros_like(img)
    for t in range(-S, S + 1):
        wt = w1[t + S]
        if t >= 0:
            tmp[:H - t] += wt * img[t:]
        else:
            tmp[-t:] += wt * img[:H + t]
    out = np.zeros_like(img)
    for t in range(-S, S + 1):
        wt = w1[t + S]
        if t >= 0:
            out[:, :W - t] += wt * tmp[:, t:]
        else:
            out[:, -t:] += wt * tmp[:, :W + t]
    return out


def spatial_filter(sigma_s, S, spatial):
    """img -> (w * img): the truncated window of radius S ("gaussian", "box"),
    or Young and van Vliet's recursive Gaussian ("recursive", S unused; see
    ``oracle.recursive``)."""
    if spatial == "recursive":
        return lambda img: recursive_gauss_2d(img, sigma_s)
    w1 = spatial_taps(sigma_s, S, spatial)
    return lambda img: conv_zero(img, w1)


def nystrom_filter(f, p, c, sigma_s, sigma_r, S, spatial="gaussian", tau=DEFAULT_TAU,
                   return_eta=False):
    """The fast filter of Section III with given landmarks ``c`` [r, D].
    ``f`` [H, W, C], ``p`` [H, W, D].  Returns g_hat [H, W, C] (and eta_hat [H, W]).

    Eq. (num1) with the range kernel replaced by the rank-r_eff expansion
    K_hat(x, y) = sum_k alpha_k v_k(x) v_k(y) of Eq. (hatK) (v_k from Eq. (vk),
    read at the guide values p(x) and p(y)).  Exchanging the window sum with
    the sum over k leaves, for every k, one spatial convolution of v_k f and
    one of v_k (Eqs. (finalnum), (finalden)):

        zeta(x) = sum_k alpha_k v_k(x) (w * (v_k f))(x),
        eta(x)  = sum_k alpha_k v_k(x) (w * v_k)(x),   g_hat = zeta / eta.
    """
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    conv = spatial_filter(sigma_s, S, spatial)
    # all extrapolated eigenvectors at once: column k of V is v_k over the pixels
    alpha, V = extrapolated_eigvecs(c, p.reshape(H * W, -1), sigma_r, tau)
    V = V.reshape(H, W, -1)
    zeta = np.zeros((H, W, C))
    eta = np.zeros((H, W))
    for k, a_k in enumerate(alpha):
        v = V[:, :, k]
        zeta += a_k * v[:, :, None] * conv(v[:, :, None] * f)
        eta += a_k * v * conv(v)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = zeta / eta[:, :, None]
    # eta_hat carries no positivity guarantee: such pixels keep f(x)
    bad = ~(eta > 0) | ~np.isfinite(eta)
    if bad.any():
        g[bad] = f[bad]
    if return_eta:
        return g, eta
    return g


def nystrom_filter_at(f, p, c, sigma_s, sigma_r, S, coords, spatial="gaussian",
                      tau=DEFAULT_TAU):
    """The same approximation evaluated pixel by pixel before the sum switch:
    Eq. (num1) with K replaced by K_hat = sum_k alpha_k v_k v_k^T (Eq. (hatK)).
    ``coords`` [M, 2] of (y, x).  Returns (g_hat [M, C], eta_hat [M])."""
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    w1 = spatial_taps(sigma_s, S, spatial)
    alpha, Wv = landmark_eig(c, sigma_r, tau)
    out = np.empty((len(coords), C))
    etas = np.empty(len(coords))
    for i, (y, x) in enumerate(np.asarray(coords)):
        ya, yb = max(0, y - S), min(H, y + S + 1)
        xa, xb = max(0, x - S), min(W, x + S + 1)
        win = p[ya:yb, xa:xb].reshape(-1, p.shape[2])
        v_win = (cross_kernel_sr(c, win, sigma_r) @ Wv) / alpha[None, :]
        v_x = (cross_kernel_sr(c, p[y, x][None, :], sigma_r) @ Wv) / alpha[None, :]
        khat = (v_win * alpha[None, :]) @ v_x[0]               # K_hat(x, y) over the window
        wsp = np.outer(w1[ya - y + S:yb - y + S], w1[xa - x + S:xb - x + S]).ravel()
        wt = wsp * khat
        eta = wt.sum()
        etas[i] = eta
        if eta > 0 and np.isfinite(eta):
            out[i] = wt @ f[ya:yb, xa:xb].reshape(-1, C) / eta
        else:
            out[i] = f[y, x]
    return out, etas


def kernel_matrix(P, sigma_r):
    """K of Eq. (kernel) on the full range list (tiny inputs only)."""
    return range_kernel_sqdist(sqdist(P, P), sigma_r)


def nystrom_kernel_matrix(P, c, sigma_r, tau=DEFAULT_TAU):
    """K_hat = sum_k alpha_k v_k v_k^T of Eq. (hatK) (tiny inputs only)."""
    alpha, V = extrapolated_eigvecs(c, P, sigma_r, tau)
    return (V * alpha[None, :]) @ V.T


def storage_error_bound(f, p, c, sigma_s, sigma_r, S, spatial="gaussian", tau=DEFAULT_TAU, center=None,
                        cross_kernel_rounding=False):
    """First-order sensitivity of g_hat(x) to a relative perturbation of every
    stored intermediate (the embedding planes u_k, the products u_k f~ and the
    convolved planes; with ``cross_kernel_rounding`` also the cross-kernel
    values b_j), used to derive per-pixel tolerances for reduced precision
    evaluations of Algorithm 1:

        B(x, c) = ( sum_k v_k(x) (w * (v_k |f~_c|))(x)
                    + |g~_c(x)| sum_k v_k(x) (w * v_k)(x) ) / |eta_hat(x)|

    with u = F^T b (u(x).u(y) = K_hat(x, y)), f~ = f - f0 and v_k = |u_k|, or
    v_k = sum_j |F_jk| b_j >= |u_k| when the b_j themselves carry a relative
    error: Eq. (vk) cancels when A is ill-conditioned, and a relative error
    delta in each b_j moves u_k by up to delta sum_j |F_jk| b_j.  A relative
    error delta in each stored value moves g_hat(x) by at most about
    delta B(x, c).  Returns B as [H, W, C]."""
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    f0 = 0.5 * (f.min(axis=(0, 1)) + f.max(axis=(0, 1))) if center is None else center
    fc = f - f0
    conv = spatial_filter(sigma_s, S, spatial)
    alpha, Wv = landmark_eig(c, sigma_r, tau)
    Fm = Wv / np.sqrt(alpha)[None, :]
    bx = cross_kernel_sr(c, p.reshape(H * W, -1), sigma_r)
    U = bx @ Fm
    Vm = bx @ np.abs(Fm) if cross_kernel_rounding else np.abs(U)
    eta = np.zeros((H, W))
    eabs = np.zeros((H, W))
    zeta = np.zeros((H, W, C))
    zabs = np.zeros((H, W, C))
    for k in range(U.shape[1]):
        uk = U[:, k].reshape(H, W)
        vk = Vm[:, k].reshape(H, W)
        eta += uk * conv(uk)
        eabs += vk * conv(vk)
        zeta += uk[:, :, None] * conv(uk[:, :, None] * fc)
        zabs += vk[:, :, None] * conv(vk[:, :, None] * np.abs(fc))
    with np.errstate(divide="ignore", invalid="ignore"):
        gt = zeta / eta[:, :, None]
        B = (zabs + np.abs(gt) * eabs[:, :, None]) / np.abs(eta)[:, :, None]
    B[~np.isfinite(B)] = np.inf
    return B


def storage_error_bound_at(f, p, c, sigma_s, sigma_r, S, coords, spatial="gaussian", tau=DEFAULT_TAU,
                           center=None):
    """``storage_error_bound`` (the |u_k| form) at the listed pixels only,
    from each pixel's window: coords [M, 2] of (y, x); ``center`` is the
    per-channel f0 (default: (min + max) / 2 of f).  Returns [M, C]."""
    f = np.asarray(f, np.float64)
    p = np.asarray(p, np.float64)
    H, W, C = f.shape
    f0 = 0.5 * (f.min(axis=(0, 1)) + f.max(axis=(0, 1))) if center is None else np.asarray(center, np.float64)
    w1 = spatial_taps(sigma_s, S, spatial)
    alpha, Wv = landmark_eig(c, sigma_r, tau)
    Fm = Wv / np.sqrt(alpha)[None, :]
    out = np.empty((len(coords), C))
    for i, (y, x) in enumerate(np.asarray(coords)):
        ya, yb = max(0, y - S), min(H, y + S + 1)
        xa, xb = max(0, x - S), min(W, x + S + 1)
        u_win = cross_kernel_sr(c, p[ya:yb, xa:xb].reshape(-1, p.shape[2]), sigma_r) @ Fm   # [n, r_eff]
        u_x = (cross_kernel_sr(c, p[y, x][None, :], sigma_r) @ Fm)[0]
        wsp = np.outer(w1[ya - y + S:yb - y + S], w1[xa - x + S:xb - x + S]).ravel()
        fc = f[ya:yb, xa:xb].reshape(-1, C) - f0
        eta = u_x @ (u_win * wsp[:, None]).sum(axis=0)
        zeta = ((u_win * wsp[:, None]) @ u_x) @ fc
        eabs = np.abs(u_x) @ (np.abs(u_win) * wsp[:, None]).sum(axis=0)
        zabs = ((np.abs(u_win) * wsp[:, None]) @ np.abs(u_x)) @ np.abs(fc)
        with np.errstate(divide="ignore", invalid="ignore"):
            out[i] = (zabs + np.abs(zeta / eta) * eabs) / abs(eta)
    out[~np.isfinite(out)] = np.inf
    return out

