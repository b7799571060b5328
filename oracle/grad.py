"""Reference gradients of the Nystrom filter.  Test infrastructure only.

The paper defines only the forward filter (Section III, Algorithm 1).  The
gradient reference is a second, independent formulation of the same
approximation written with torch float64 CPU ops so that autograd supplies
the derivatives:

* b_k(x) = k(c_k, p(x)) = exp(-|p(x) - c_k|^2 / (2 sigma_r^2))   (Eq. (defB))
* M^{1/2} = A^{-1/2} from the eigendecomposition of A (Eqs. (defA), (eigA));
  u(x) = M^{1/2} b(x), so u(x).u(y) = b(x)^T A^{-1} b(y) = K_hat(x, y), the
  same low-rank kernel as Eq. (hatK) with the v_k of Eq. (vk)
* Z_kc = w * (u_k f_c), E_k = w * u_k with the separable spatial kernel
  w1(t) = exp(-t^2 / (2 sigma_s^2)) on [-S, S] (window radius S held fixed)
* zeta_c = sum_k u_k Z_kc, eta = sum_k u_k E_k, g = zeta / eta.

Landmarks are constants.  ``central_difference`` gives the finite-difference
check (h = 1e-3 by default).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def _conv_sep_zero(X, w1):
    """Separable zero-padded correlation of every plane of X [P, H, W]."""
    S = (w1.numel() - 1) // 2
    P = X.shape[0]
    x = X.unsqueeze(0)
    kr = w1.view(1, 1, -1, 1).expand(P, 1, -1, 1)
    kc = w1.view(1, 1, 1, -1).expand(P, 1, 1, -1)
    x = F.conv2d(x, kr, padding=(S, 0), groups=P)
    x = F.conv2d(x, kc, padding=(0, S), groups=P)
    return x[0]


def nystrom_torch(f, p, c, sigma_s, sigma_r, S, spatial="gaussian"):
    """Differentiable float64 Nystrom filter.  ``f`` [H, W, C], ``p`` [H, W, D],
    ``c`` [r, D], ``sigma_s`` and ``sigma_r`` 0-d tensors.  Returns g [H, W, C]."""
    H, W, C = f.shape
    D = p.shape[2]
    P = p.reshape(H * W, D)
    dcc = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    A = torch.exp(-dcc / (2.0 * sigma_r ** 2))
    lam, Q = torch.linalg.eigh(A)
    Mh = (Q * lam.rsqrt()[None, :]) @ Q.T
    d2 = ((P[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    b = torch.exp(-d2 / (2.0 * sigma_r ** 2))
    u = b @ Mh                                            # [N, r]
    t = torch.arange(-S, S + 1, dtype=torch.float64)
    if spatial == "gaussian":
        w1 = torch.exp(-(t * t) / (2.0 * sigma_s ** 2))
    else:
        w1 = torch.ones_like(t)
    r = c.shape[0]
    U = u.T.reshape(r, H, W)
    fc = f.permute(2, 0, 1)                                # [C, H, W]
    planes = torch.cat([U[:, None] * fc[None], U[:, None]], dim=1)   # [r, C+1, H, W]
    Zs = _conv_sep_zero(planes.reshape(r * (C + 1), H, W), w1).reshape(r, C + 1, H, W)
    contr = (U[:, None] * Zs).sum(0)                      # [C+1, H, W]
    g = contr[:C] / contr[C][None]
    return g.permute(1, 2, 0)


def reference_grads(f, p, c, sigma_s, sigma_r, S, G, spatial="gaussian"):
    """Gradients of L = sum(G * g) w.r.t. f, p, sigma_r, sigma_s (float64)."""
    ft = torch.tensor(np.asarray(f, np.float64), requires_grad=True)
    pt = torch.tensor(np.asarray(p, np.float64), requires_grad=True)
    ct = torch.tensor(np.asarray(c, np.float64))
    ss = torch.tensor(float(sigma_s), dtype=torch.float64, requires_grad=True)
    sr = torch.tensor(float(sigma_r), dtype=torch.float64, requires_grad=True)
    g = nystrom_torch(ft, pt, ct, ss, sr, S, spatial)
    L = (g * torch.tensor(np.asarray(G, np.float64))).sum()
    L.backward()
    return dict(g=g.detach().numpy(), f=ft.grad.numpy(), p=pt.grad.numpy(),
                sigma_r=float(sr.grad), sigma_s=float(ss.grad) if spatial == "gaussian" else 0.0)


def central_difference(fn, x0, h=1e-3):
    """(fn(x0 + h) - fn(x0 - h)) / (2h) for a scalar function of a scalar."""
    return (fn(x0 + h) - fn(x0 - h)) / (2.0 * h)
